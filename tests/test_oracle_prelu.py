"""Pins of the oracle's PReLU network (§3 Eq. 2 and 3), each against
something other than the oracle's own formula: a hand-computed tiny network,
the affine special case (slopes 1) composed with numpy matrix products,
positive homogeneity of a bias-free network, central finite differences of
the loss, the parameter count in closed form, and the bf16 emulation within
its rounding bound."""
import numpy as np
import pytest

UNIT_NORM = np.array([0.0] * 6 + [1.0] * 6 + [0.0] * 6 + [1.0] * 6)


def layout(orc, sh, p):
    """Split the flat parameters into (A, b, slope) per layer (slope None for the output)."""
    out, off = [], 0
    for l in range(sh.hidden + 1):
        ni = 6 if l == 0 else sh.width
        no = 6 if l == sh.hidden else sh.width
        A = p[off:off + no * ni].reshape(no, ni)
        off += no * ni
        b = p[off:off + no]
        off += no
        a = None
        if l < sh.hidden:
            a = p[off]
            off += 1
        out.append((A, b, a))
    assert off == len(p)
    return out


def test_nparams_closed_form(orc):
    for W, H in [(700, 3), (900, 5), (2, 1), (64, 2)]:
        sh = orc.shape(width=W, hidden=H)
        assert orc.prelu_nparams(sh) == 6 * W + W + 1 + (H - 1) * (W * W + W + 1) + 6 * W + 6


def test_init_slopes_and_bounds(orc):
    sh = orc.shape(width=50, hidden=3)
    p = orc.prelu_init(sh, 11)
    for l, (A, b, a) in enumerate(layout(orc, sh, p)):
        bound = 1 / np.sqrt(6 if l == 0 else 50)
        assert np.abs(A).max() <= bound and np.abs(b).max() <= bound
        assert np.abs(A).max() > 0.8 * bound
        assert a is None or a == np.float32(0.25)


def test_hand_computed_tiny_network(orc):
    # width 2, one hidden layer; normalised input (1, -2, 0.5, 0, 0, 3)
    # v = (1 + 0.5, -2 + 0.25) = (1.5, -1.75); h = (1.5, 0.25 * -1.75 = -0.4375)
    # y = (h0, h1, h0 + h1, 2 h0, -h1, 1) = (1.5, -0.4375, 1.0625, 3.0, 0.4375, 1.0)
    sh = orc.shape(width=2, hidden=1)
    A0 = np.zeros((2, 6)); A0[0, 0] = 1; A0[1, 1] = 1
    A1 = np.array([[1, 0], [0, 1], [1, 1], [2, 0], [0, -1], [0, 0]], dtype=float)
    p = np.concatenate([A0.ravel(), [0.5, 0.25], [0.25], A1.ravel(), [0, 0, 0, 0, 0, 1]]).astype(np.float32)
    x = np.array([[1.0], [-2.0], [0.5], [0.0], [0.0], [3.0]])
    for mode in (0, 1):
        y = orc.prelu_apply(sh, p, UNIT_NORM, x, mode=mode)
        assert np.array_equal(y[:, 0], [1.5, -0.4375, 1.0625, 3.0, 0.4375, 1.0])
    # a non-unit normalisation: input (x - mu)/sd, output mu + sd y
    norm = UNIT_NORM.copy()
    norm[0:6] = 1.0; norm[6:12] = 2.0; norm[12:18] = -1.0; norm[18:24] = 4.0
    y = orc.prelu_apply(sh, p, norm, 1.0 + 2.0 * x, mode=0)
    assert np.allclose(y[:, 0], -1.0 + 4.0 * np.array([1.5, -0.4375, 1.0625, 3.0, 0.4375, 1.0]), rtol=0, atol=1e-15)


def test_unit_slopes_give_the_composed_affine_map(orc):
    sh = orc.shape(width=40, hidden=4)
    p = orc.prelu_init(sh, 3).copy()
    layers = layout(orc, sh, p)
    for l in range(sh.hidden):
        off = sum(A.size + b.size + 1 for A, b, _ in layers[:l]) + layers[l][0].size + layers[l][1].size
        p[off] = 1.0
    layers = layout(orc, sh, p)
    M, c = np.eye(6), np.zeros(6)
    for A, b, _ in layers:                  # compose first, apply once
        M, c = A.astype(float) @ M, A.astype(float) @ c + b
    x = np.random.default_rng(0).normal(size=(6, 200))
    y = orc.prelu_apply(sh, p, UNIT_NORM, x, mode=0)
    assert np.allclose(y, M @ x + c[:, None], rtol=0, atol=1e-12)


def test_bias_free_network_is_positively_homogeneous(orc):
    sh = orc.shape(width=30, hidden=3)
    p = orc.prelu_init(sh, 4).copy()
    off = 0
    for l, (A, b, a) in enumerate(layout(orc, sh, p)):
        off += A.size
        p[off:off + b.size] = 0
        off += b.size + (a is not None)
    x = np.random.default_rng(1).normal(size=(6, 100))
    y1 = orc.prelu_apply(sh, p, UNIT_NORM, x, mode=0)
    y3 = orc.prelu_apply(sh, p, UNIT_NORM, 3.0 * x, mode=0)
    assert np.allclose(y3, 3.0 * y1, rtol=1e-13, atol=1e-14)
    yn = orc.prelu_apply(sh, p, UNIT_NORM, -x, mode=0)
    assert not np.allclose(yn, -y1)         # not odd: the slope 0.25 bites


def test_gradient_matches_central_differences(orc):
    sh = orc.shape(width=12, hidden=3)
    rng = np.random.default_rng(2)
    p = orc.prelu_init(sh, 9).astype(np.float64)
    zin = rng.normal(size=(6, 40))
    zout = rng.normal(size=(6, 40))
    idx = np.arange(40)
    norm = UNIT_NORM

    # the oracle takes FP32 parameters: probe with steps that FP32 represents exactly
    def loss_at(q):
        return orc.prelu_loss_grad(sh, q.astype(np.float32), norm, zin, zout, idx)[0]

    _, g = orc.prelu_loss_grad(sh, p.astype(np.float32), norm, zin, zout, idx)
    layers = layout(orc, sh, p)
    picks = list(rng.choice(len(p), 60, replace=False))
    off = 0
    for A, b, a in layers:                  # every slope, too
        off += A.size + b.size
        if a is not None:
            picks.append(off)
            off += 1
    for k in picks:
        h = 2.0 ** -10
        qp, qm = p.copy(), p.copy()
        qp[k] += h
        qm[k] -= h
        fd = (loss_at(qp) - loss_at(qm)) / (2 * h)
        assert fd == pytest.approx(g[k], rel=2e-3, abs=1e-7), k


def test_bf16_emulation_within_rounding_bound(orc):
    sh = orc.shape(width=100, hidden=3)
    p = orc.prelu_init(sh, 5)
    x = np.random.default_rng(3).normal(size=(6, 300))
    y0 = orc.prelu_apply(sh, p, UNIT_NORM, x, mode=0)
    y1 = orc.prelu_apply(sh, p, UNIT_NORM, x, mode=1)
    d = np.abs(y1 - y0) / np.abs(y0).std(axis=1, keepdims=True)
    # bf16 keeps 8 significant bits: each product of a rounded weight and a
    # rounded activation is off by up to ~2^-8 relative, independently, so an
    # output's sum over a layer is off by ~2^-8 of its spread per layer and the
    # four layers add in quadrature: ~8e-3 typical, a few times that at the
    # tails of 1800 outputs.
    assert d.max() < 6e-2 and np.median(d) < 1e-2 and d.max() > 0
