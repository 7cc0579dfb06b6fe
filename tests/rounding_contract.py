"""The documented arithmetic of the library's tanh surrogate kernels, as the
rounding points of oracle.mlp_error.Rounding (the header states them: bf16
weights and activations in the hidden and output layers, 16 significant bits
in the first layer, FP32 sums, FP32 output, tanh to 2^-20 absolute, bf16
back-propagated errors in training).  The GPU parity tests compare the
library with the FP64 network and allow what these rounding points allow."""
from oracle import mlp_error as me

BF16 = 2.0 ** -8           # unit roundoff: 8 significant bits
SPLIT16 = 2.0 ** -15       # hi + lo bf16 pair: 16 bits, less the dropped lo*lo term
FP32 = 2.0 ** -24

# 70 terms: 64 products + bias, rounded up
SURROGATE = me.Rounding(u_w=[SPLIT16, BF16, BF16, BF16], u_x=[SPLIT16, BF16, BF16, BF16],
                        e_act=2.0 ** -20, u_acc=70 * FP32, u_out=FP32, u_d=BF16)

# Hoeffding: P(|E| >= LAM * S) <= 2 exp(-LAM^2 / 2) = 4.6e-11 per output
LAM = 7.0
