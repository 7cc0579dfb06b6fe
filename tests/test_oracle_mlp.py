"""Pins of the oracle's surrogate network (CPU only): Eq. (3) forward, Eq. (4)
MSE and its reverse-mode gradient, Adam, bf16 rounding, and training."""
import math

import numpy as np
import pytest

X, Y, T, PX, PY, PT = range(6)


def bf16_by_definition(x32):
    """Nearest bfloat16 (8 significant bits) with ties to even, by comparing
    the two neighbouring candidates exactly in float64."""
    out = np.empty_like(x32)
    bits = x32.view(np.uint32)
    lo = (bits & np.uint32(0xFFFF0000)).view(np.float32)
    hi_bits = (bits & np.uint32(0xFFFF0000)) + np.uint32(0x10000)
    hi = hi_bits.view(np.float32)
    x = x32.astype(np.float64)
    dlo = np.abs(x - lo.astype(np.float64))
    dhi = np.abs(hi.astype(np.float64) - x)
    lo_even = ((bits >> np.uint32(16)) & np.uint32(1)) == 0
    pick_lo = (dlo < dhi) | ((dlo == dhi) & lo_even)
    out[:] = np.where(pick_lo, lo, hi)
    return out


def test_bf16_round_to_nearest_even(orc):
    hi = np.arange(0, 1 << 16, dtype=np.uint32) << np.uint32(16)
    low = np.array([0, 1, 0x7FFF, 0x8000, 0x8001, 0xFFFF, 0x1234, 0xC000], dtype=np.uint32)
    bits = (hi[:, None] | low[None, :]).ravel()
    x = bits.view(np.float32)
    finite = np.isfinite(x) & (np.abs(x) < np.float32(3.38e38))
    x = x[finite]
    import ctypes as C
    f = orc.lib().orc_bf16
    sample = x[:: 7]
    got = np.array([f(float(v)) for v in sample], dtype=np.float32)
    want = bf16_by_definition(sample)
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))


def make_pairs(orc, n, seed=5):
    zin = orc.fill_gaussian(n, seed, sigma=(1e-5, 1e-5, 1e-5, 1e-4, 1e-4, 1e-3))
    zout = zin.copy()
    zout[X] = zin[X] * 0.3 + 2e-2 * zin[PX] + 1e3 * zin[X] * zin[PT]
    zout[PX] = -zin[X] * 2.0 + 0.1 * zin[PX] + 3e-3 * np.tanh(zin[PT] * 1e3)
    zout[Y] = zin[Y] + 0.1 * zin[PY]
    return np.ascontiguousarray(zin), np.ascontiguousarray(zout)


def bf16_exact_params(orc, sh, seed):
    """Initial parameters rounded to bf16: perturbations by 2^-10 stay exact in FP32."""
    p = orc.mlp_init(sh, seed)
    return orc.bf16(p)


@pytest.mark.parametrize("hidden,width", [(3, 16), (1, 8), (0, 4)])
def test_gradient_vs_finite_differences(orc, hidden, width):
    sh = orc.shape(6, width, hidden, 6)
    zin, zout = make_pairs(orc, 64)
    norm = orc.norm_stats(zin, zout, 64)
    p = bf16_exact_params(orc, sh, 3)
    idx = np.arange(0, 64, 3)
    _, g = orc.mlp_loss_grad(sh, p, norm, zin, zout, idx, mode=0)
    rng = np.random.default_rng(0)
    picks = rng.choice(len(p), size=min(40, len(p)), replace=False)
    h = 2.0 ** -10

    def D(k, hh):
        a = p.copy(); a[k] += np.float32(hh)
        b = p.copy(); b[k] -= np.float32(hh)
        assert float(a[k]) - float(p[k]) == hh and float(p[k]) - float(b[k]) == hh
        la, _ = orc.mlp_loss_grad(sh, a, norm, zin, zout, idx, mode=0)
        lb, _ = orc.mlp_loss_grad(sh, b, norm, zin, zout, idx, mode=0)
        return (la - lb) / (2 * hh)

    gmax = np.abs(g).max()
    for k in picks:
        fd = (4 * D(k, h / 2) - D(k, h)) / 3          # Richardson: O(h^4)
        assert abs(fd - g[k]) <= 1e-7 * max(abs(g[k]), 1e-3 * gmax)


def test_adam_first_step_closed_form(orc):
    """At t = 1 the bias-corrected moments are g and g^2: step = -lr g/(|g| + eps)."""
    rng = np.random.default_rng(1)
    p = rng.normal(size=50).astype(np.float32)
    g = rng.normal(size=50) * 10.0 ** rng.uniform(-6, 1, 50)
    p1, m, v = orc.adam_step(p, np.zeros(50), np.zeros(50), g, 1, lr=1e-3)
    want = p.astype(np.float64) - 1e-3 * g / (np.abs(g) + 1e-8)
    assert np.allclose(p1, want.astype(np.float32), rtol=0, atol=1e-7)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_linear_model_trains_to_least_squares(orc):
    """No hidden layer: the MSE minimiser is the least-squares affine fit in
    normalised coordinates (normal equations)."""
    sh = orc.shape(6, 4, 0, 6)
    zin, zout = make_pairs(orc, 1000, seed=8)
    p0 = orc.mlp_init(sh, 1)
    p, norm, log = orc.mlp_train(sh, p0, zin, zout, batch=700, epochs=3000, lr=1e-2,
                                 train_frac=0.7, shuffle_seed=4, mode=0)
    ntr = 700
    xh = (zin[:, :ntr] - norm[0:6, None]) / norm[6:12, None]
    yh = (zout[:, :ntr] - norm[12:18, None]) / norm[18:24, None]
    Amat = np.vstack([xh, np.ones(ntr)]).T
    sol, *_ = np.linalg.lstsq(Amat, yh.T, rcond=None)
    W = p[:36].reshape(6, 6).astype(np.float64)
    b = p[36:42].astype(np.float64)
    assert np.abs(W - sol[:6].T).max() < 2e-3
    assert np.abs(b - sol[6]).max() < 2e-3
    assert log[-1, 0] < log[0, 0]


def test_bf16_mode_tracks_fp64_mode(orc):
    sh = orc.shape()
    zin, zout = make_pairs(orc, 512)
    norm = orc.norm_stats(zin, zout, 512)
    p = orc.mlp_init(sh, 7)
    y0 = orc.mlp_apply(sh, p, norm, zin, mode=0)
    y1 = orc.mlp_apply(sh, p, norm, zin, mode=1)
    d = np.abs(y1 - y0) / norm[18:24, None]
    assert d.max() < 3e-2 and d.mean() < 5e-3
    _, g0 = orc.mlp_loss_grad(sh, p, norm, zin, zout, np.arange(256), mode=0)
    _, g1 = orc.mlp_loss_grad(sh, p, norm, zin, zout, np.arange(256), mode=1)
    assert np.linalg.norm(g1 - g0) / np.linalg.norm(g0) < 3e-2


def test_training_reduces_test_loss(orc):
    sh = orc.shape(6, 16, 2, 6)
    zin, zout = make_pairs(orc, 4000, seed=9)
    p0 = orc.mlp_init(sh, 2)
    p, norm, log = orc.mlp_train(sh, p0, zin, zout, batch=256, epochs=8, lr=3e-3, mode=1,
                                 shuffle_seed=1)
    assert log[-1, 1] < 0.5 * log[0, 1]
    assert np.all(np.isfinite(log))
