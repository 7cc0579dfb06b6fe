"""Rounding-error models of the surrogate network -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
module; the product path never does.

The network is the feed-forward map of the paper's §3 Eq. (3) with tanh,
F = L_3 o tanh o L_2 o tanh o L_1 o tanh o L_0 on the coordinates normalised
per direction (§3), trained on the mean-squared error of Eq. (4).  This
module evaluates it, and its loss gradient, a second time, in plain numpy
FP64 (vectorised over particles, independent of the C oracle's per-particle
loops; the tests require the two to agree), and then asks how far a
reduced-precision implementation of it may land from the FP64 values.

An implementation is described by its ROUNDING POINTS -- the operands it
rounds and the unit roundoff of each -- as a :class:`Rounding` record:

* ``u_w[l]``: the weights of layer l as they enter its product,
* ``u_x[l]``: the input of layer l (the normalised coordinates for l = 0, the
  hidden activation tanh(a_{l-1}) otherwise) as it enters the product,
* ``e_act``: absolute error of one tanh evaluation,
* ``u_acc``: relative error of one accumulated dot product, applied to the
  sum of the absolute values of its terms (n u for an n-term sum in a
  format of unit roundoff u),
* ``u_out``: the stored output,
* ``u_d``: back-propagated errors of layers >= 1 entering products.

A value v rounded with unit roundoff u becomes v (1 + d), |d| <= u (round to
nearest; bfloat16 keeps 8 significant bits, u = 2^-8; FP32 24, u = 2^-24).

Two uses:

* :func:`forward_bound` -- a first-order a-priori bound and a probabilistic
  scale, per output and particle.  To first order the output error is a sum
  E_j = sum_k J_jk d_k v_k over all rounding points k, J_jk the derivative of
  output j with respect to the value v_k, computed here by back-propagating
  each output through the FP64 network.  Hence
    |E_j| <= B_j = sum_k |J_jk| u_k |v_k|                (worst case),
  and if the d_k behave as independent, mean-zero and bounded by u_k (the
  random model of rounding of Higham and Mary, SIAM J. Sci. Comput. 41,
  2019), Hoeffding's inequality gives
    P(|E_j| >= lam S_j) <= 2 exp(-lam^2 / 2),  S_j = sqrt(sum_k (J_jk u_k v_k)^2).
  The weights' rounding is shared by all particles, so over particles the
  E_j are correlated; for each one the bound holds as stated.

* :func:`perturbed_forward` / :func:`loss_grad` with ``rng`` -- Monte-Carlo
  arithmetic (D. S. Parker, "Monte Carlo Arithmetic", UCLA CSD-970002, 1997):
  every rounding point applies v (1 + u xi), xi uniform on [-1, 1], drawn
  independently per value (a weight's draw is shared by all particles of one
  pass, as a weight is rounded once).  The spread of an ensemble of such
  passes measures how far a result computed with those rounding points may
  move; the tests use it for the loss gradient, whose first-order analysis
  would need second derivatives.

Normalised units throughout: output j in units of the training output's
standard deviation sd_out[j] (norm[18 + j]).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

N_IN, N_OUT = 6, 6


@dataclass
class Rounding:
    """Unit roundoff of each rounding point (see the module docstring)."""
    u_w: Sequence[float]
    u_x: Sequence[float]
    e_act: float = 0.0
    u_acc: float = 0.0
    u_out: float = 0.0
    u_d: float = 0.0


@dataclass
class Net:
    """Weights A_l (out x in) and biases b_l of layers 0..H, FP64."""
    A: List[np.ndarray] = field(default_factory=list)
    b: List[np.ndarray] = field(default_factory=list)

    @property
    def H(self) -> int:
        return len(self.A) - 1


def unpack(params: np.ndarray, width: int, hidden: int) -> Net:
    """Flat FP32 parameters A_0, b_0, A_1, b_1, ..., A_H, b_H (row-major
    [out][in] weights), the layout of the library and the C oracle."""
    p = np.asarray(params, dtype=np.float64)
    net = Net()
    off = 0
    for l in range(hidden + 1):
        ni = N_IN if l == 0 else width
        no = N_OUT if l == hidden else width
        net.A.append(p[off:off + no * ni].reshape(no, ni))
        off += no * ni
        net.b.append(p[off:off + no].copy())
        off += no
    if off != p.size:
        raise ValueError(f"{p.size} parameters, the shape needs {off}")
    return net


def normalise_in(zin: np.ndarray, norm: np.ndarray) -> np.ndarray:
    """(6, n) raw bunch -> (n, 6) network input (x - mu_in) / sd_in (§3)."""
    return ((zin - norm[0:6, None]) / norm[6:12, None]).T


def normalise_out(zout: np.ndarray, norm: np.ndarray) -> np.ndarray:
    return ((zout - norm[12:18, None]) / norm[18:24, None]).T


def _perturb(v, u, rng):
    if rng is None or u == 0.0:
        return v
    return v * (1.0 + u * rng.uniform(-1.0, 1.0, size=np.shape(v)))


def perturbed_forward(net: Net, x: np.ndarray, rnd: Optional[Rounding] = None, rng=None):
    """Network of Eq. (3) on the (n, 6) normalised inputs x.  Returns the
    inputs of every layer as used (hs[0..H]), the pre-activations (a[0..H]) and
    the output (= a[H] after output rounding).  With rnd and rng, each rounding
    point is perturbed at random (Monte-Carlo arithmetic)."""
    H = net.H
    hs, pre = [], []
    h = x
    for l in range(H + 1):
        if rnd is not None:
            h = _perturb(h, rnd.u_x[l], rng)
        hs.append(h)
        A = net.A[l] if rnd is None else _perturb(net.A[l], rnd.u_w[l], rng)
        a = h @ A.T + net.b[l]
        if rnd is not None and rng is not None and rnd.u_acc:
            a = a + rnd.u_acc * (np.abs(h) @ np.abs(A).T + np.abs(net.b[l])) * rng.uniform(-1, 1, a.shape)
        pre.append(a)
        if l < H:
            h = np.tanh(a)
            if rnd is not None and rng is not None and rnd.e_act:
                h = h + rnd.e_act * rng.uniform(-1, 1, h.shape)
    y = pre[H] if rnd is None else _perturb(pre[H], rnd.u_out, rng)
    return hs, pre, y


def forward(net: Net, x: np.ndarray) -> np.ndarray:
    return perturbed_forward(net, x)[2]


def loss_grad(net: Net, x: np.ndarray, yt: np.ndarray, rnd: Optional[Rounding] = None, rng=None):
    """MSE of Eq. (4) over the batch (mean over samples and the 6 outputs) and
    its gradient by reverse-mode differentiation, as a flat FP64 vector in the
    parameter layout of :func:`unpack`.  With rnd and rng the forward is
    perturbed as in :func:`perturbed_forward`, and the back-propagated errors
    of layers >= 1 (rnd.u_d) and the weights they meet (rnd.u_w, a separate
    draw: a transposed copy is rounded on its own) as well."""
    H = net.H
    hs, pre, y = perturbed_forward(net, x, rnd, rng)
    B = x.shape[0]
    r = y - yt
    loss = float(np.mean(r * r))
    delta = r * (2.0 / (B * N_OUT))            # dL/da_H
    grads_A, grads_b = [None] * (H + 1), [None] * (H + 1)
    for l in range(H, -1, -1):
        grads_b[l] = delta.sum(axis=0)
        d = delta if (rnd is None or l == 0) else _perturb(delta, rnd.u_d, rng)
        grads_A[l] = d.T @ hs[l]
        if l > 0:
            A = net.A[l] if rnd is None else _perturb(net.A[l], rnd.u_w[l], rng)
            e = d @ A
            delta = e * (1.0 - hs[l] * hs[l])
    flat = []
    for l in range(H + 1):
        flat.append(grads_A[l].ravel())
        flat.append(grads_b[l])
    return loss, np.concatenate(flat)


def forward_bound(net: Net, x: np.ndarray, rnd: Rounding):
    """First-order worst-case bound B and probabilistic scale S (both (n, 6),
    normalised units) of the output error of an implementation with the
    rounding points rnd, at the FP64 network values (module docstring)."""
    H = net.H
    hs, pre, y = perturbed_forward(net, x)
    n = x.shape[0]
    # J[l] = d y / d a_l, shape (n, 6, width_l), by back-propagation of each output
    J = [None] * (H + 1)
    J[H] = np.broadcast_to(np.eye(N_OUT), (n, N_OUT, N_OUT))
    for l in range(H, 0, -1):
        dh = J[l] @ net.A[l]                                   # d y / d h_l
        J[l - 1] = dh * (1.0 - hs[l] * hs[l])[:, None, :]
    Bw = np.zeros((n, N_OUT))
    S2 = np.zeros((n, N_OUT))
    for l in range(H + 1):
        absA = np.abs(net.A[l])
        ah = np.abs(hs[l])
        row = ah @ absA.T                                      # sum_i |A_oi h_i|, (n, out)
        aJ = np.abs(J[l])
        # weight rounding: term k = (o, i), J = J_l[o] h_i, value A_oi
        Bw += np.einsum("njo,no->nj", aJ, rnd.u_w[l] * row)
        S2 += np.einsum("njo,no->nj", J[l] ** 2, (rnd.u_w[l] ** 2) * ((ah * ah) @ (absA * absA).T))
        # accumulation: |J_l[o]| u_acc (sum_i |A_oi h_i| + |b_o|)
        Bw += np.einsum("njo,no->nj", aJ, rnd.u_acc * (row + np.abs(net.b[l])))
        # input operand rounding and (l >= 1) tanh evaluation: d y / d h_l
        dh = J[l] @ net.A[l]
        Bw += (np.abs(dh) * (rnd.u_x[l] * ah)[:, None, :]).sum(-1)
        S2 += ((dh * (rnd.u_x[l] * ah)[:, None, :]) ** 2).sum(-1)
        if l > 0 and rnd.e_act:
            Bw += rnd.e_act * np.abs(dh).sum(-1)
            S2 += (rnd.e_act ** 2) * (dh ** 2).sum(-1)
    Bw += rnd.u_out * np.abs(y)
    S2 += (rnd.u_out * y) ** 2
    return y, Bw, np.sqrt(S2)
