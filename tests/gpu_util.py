"""Helpers for the GPU parity tests: host<->device bunch copies and the parity
metric.  No computation of the method happens here."""
import numpy as np

X, Y, T, PX, PY, PT = range(6)


def torch_mod():
    import torch
    return torch


def to_dev(z_np):
    """(6, n) numpy FP64 -> (6, ld) device tensor with even ld."""
    torch = torch_mod()
    n = z_np.shape[1]
    ld = n + (n & 1)
    t = torch.zeros((6, max(ld, 2)), dtype=torch.float64, device="cuda")
    if n:
        t[:, :n] = torch.from_numpy(np.ascontiguousarray(z_np)).cuda()
    return t


def to_host(t, n):
    torch = torch_mod()
    torch.cuda.synchronize()
    return np.ascontiguousarray(t[:, :n].cpu().numpy())


def rel_err(g, c, cols=None):
    """Per coordinate j: max_i |g_ij - c_ij| / max(|c_ij|, rms_j(c))."""
    if cols is not None:
        g = g[:, cols]
        c = c[:, cols]
    rms = np.sqrt(np.mean(c * c, axis=1))[:, None]
    den = np.maximum(np.abs(c), rms)
    den[den == 0] = 1.0
    return (np.abs(g - c) / den).max(axis=1)
