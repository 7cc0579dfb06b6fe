"""Pins of the oracle's tanh surrogate network (§3 Eq. 3 and 4) against facts
that do not come from the oracle itself, and of its rounding-error models:

* a two-hidden-layer network whose pre-activations are chosen so that the
  hidden values are known in closed form (tanh(ln 2) = 3/5, tanh(ln 3 / 2) =
  1/2, then tanh 1 and tanh 1/2 through exp), evaluated by hand;
* a probe of the flat parameter layout: in a network whose deeper layers are
  selection matrices, perturbing one parameter moves exactly the outputs its
  (layer, row, column) reaches;
* the second, vectorised numpy evaluation of the network and its gradient
  agrees with the C oracle's per-particle loops;
* the first-order error bound covers an actual bf16 implementation of the
  network (the oracle's kernel-emulating mode), and its probabilistic scale
  agrees with the spread of a Monte-Carlo-arithmetic ensemble;
* Philox4x32-10 against the published known-answer vectors;
* the learning-rate schedule's defining properties."""
import math
import os

import numpy as np
import pytest

from oracle import mlp_error as me

HERE = os.path.dirname(os.path.abspath(__file__))


def tiny_shape(orc):
    return orc.shape(6, 2, 2, 6)


# normalisation of the hand-computed network: raw = mu + sd * normalised
MU_IN = np.array([0.5, -0.25, 1.0, 2.0, -1.0, 0.125])
SD_IN = np.array([2.0, 0.5, 4.0, 1.0, 8.0, 0.25])
MU_OUT = np.array([1e-6, -2e-6, 3e-6, 1e-4, -1e-4, 5e-4])
SD_OUT = np.array([1e-5, 2e-5, 1e-5, 1e-4, 2e-4, 1e-3])
A0 = np.array([[1.0, 2.0, -1.0, 0.5, 0.25, -2.0], [-0.5, 1.0, 3.0, -1.0, 0.5, 4.0]])
B0 = np.array([0.375, -0.75])
A1 = np.array([[5.0, 2.0], [-5.0, 4.0]])
B1 = np.array([-3.0, 1.5])
A2 = np.array([[1.0, -1.0], [2.0, 0.5], [-0.25, 3.0], [0.75, -1.5], [-2.0, -0.5], [4.0, 1.0]])
B2 = np.array([0.5, -1.0, 0.25, 2.0, -0.125, 0.0])


def hand_network():
    """Flat parameters (A_0, b_0, A_1, b_1, A_2, b_2), normalisation, and a raw
    input whose normalised coordinates make the first pre-activations ln 2 and
    ln(3)/2: x_2..x_5 are fixed and x_0, x_1 solve the two linear equations."""
    params = np.concatenate([A0.ravel(), B0, A1.ravel(), B1, A2.ravel(), B2]).astype(np.float32)
    assert np.array_equal(params.astype(np.float64),
                          np.concatenate([A0.ravel(), B0, A1.ravel(), B1, A2.ravel(), B2]))  # FP32-exact
    xt = np.array([0.0, 0.0, 0.25, -0.5, 1.0, 0.125])
    rest = A0[:, 2:] @ xt[2:] + B0
    target = np.array([math.log(2.0), 0.5 * math.log(3.0)])
    xt[:2] = np.linalg.solve(A0[:, :2], target - rest)
    raw = MU_IN + SD_IN * xt
    norm = np.concatenate([MU_IN, SD_IN, MU_OUT, SD_OUT])
    return params, norm, raw


def test_hand_computed_two_hidden_layers(orc):
    """h1 = (tanh ln 2, tanh(ln 3 / 2)) = (3/5, 1/2); a1 = A1 h1 + b1 = (1, 1/2);
    h2 = ((e^2 - 1)/(e^2 + 1), (e - 1)/(e + 1)); y = A2 h2 + b2, no activation on
    the output layer; the stored output is mu_out + sd_out y."""
    params, norm, raw = hand_network()
    e = math.e
    h2 = np.array([(e * e - 1.0) / (e * e + 1.0), (e - 1.0) / (e + 1.0)])
    assert np.allclose(A1 @ np.array([0.6, 0.5]) + B1, [1.0, 0.5], rtol=0, atol=1e-15)
    y = A2 @ h2 + B2
    want = MU_OUT + SD_OUT * y
    z = np.ascontiguousarray(np.tile(raw[:, None], (1, 3)))
    got = orc.mlp_apply(tiny_shape(orc), params, norm, z, mode=0)
    for k in range(3):
        assert np.allclose(got[:, k], want, rtol=1e-14, atol=0), (got[:, k], want)
    # the numpy evaluation agrees with the hand values as well
    yn = me.forward(me.unpack(params, 2, 2), me.normalise_in(z, norm))
    assert np.allclose(yn[0], y, rtol=1e-14, atol=1e-15)


def test_hand_computed_loss(orc):
    """Eq. (4): mean over the batch and the six outputs of the squared
    normalised error; with target y + r for a chosen r the loss is mean(r^2)."""
    params, norm, raw = hand_network()
    e = math.e
    y = A2 @ np.array([(e * e - 1.0) / (e * e + 1.0), (e - 1.0) / (e + 1.0)]) + B2
    r = np.array([0.5, -0.25, 1.0, 0.0, -2.0, 0.125])
    zin = np.ascontiguousarray(np.tile(raw[:, None], (1, 2)))
    zout = np.ascontiguousarray(np.tile((MU_OUT + SD_OUT * (y + r))[:, None], (1, 2)))
    loss, _ = orc.mlp_loss_grad(tiny_shape(orc), params, norm, zin, zout, np.array([0, 1]), mode=0)
    assert abs(loss - np.mean(r * r)) <= 1e-14 * np.mean(r * r)


def selection_network(orc, rng):
    """Width 8, two hidden layers: A_0 dense, A_1 = 0.5 x a permutation
    (unit o reads unit P1[o]), A_2 selects output j = unit P2[j]."""
    W, P1, P2 = 8, [5, 2, 7, 0, 3, 6, 1, 4], [3, 0, 6, 1, 7, 4]
    A0_ = rng.uniform(-1, 1, (W, 6))
    b0 = rng.uniform(-0.5, 0.5, W)
    A1_ = np.zeros((W, W))
    for o, i in enumerate(P1):
        A1_[o, i] = 0.5
    b1 = rng.uniform(-0.5, 0.5, W)
    A2_ = np.zeros((6, W))
    for j, i in enumerate(P2):
        A2_[j, i] = 1.0
    b2 = rng.uniform(-0.5, 0.5, 6)
    p = np.concatenate([A0_.ravel(), b0, A1_.ravel(), b1, A2_.ravel(), b2]).astype(np.float32)
    return p, P1, P2


def reached_outputs(p_index, P1, P2):
    """Outputs that parameter p_index can move, from the documented layout
    (A_0 8x6, b_0 8, A_1 8x8, b_1 8, A_2 6x8, b_2 6; weights row-major [out][in])."""
    W = 8
    sizes = [("A0", W * 6), ("b0", W), ("A1", W * W), ("b1", W), ("A2", 6 * W), ("b2", 6)]
    off = 0
    for name, size in sizes:
        if p_index < off + size:
            q = p_index - off
            break
        off += size
    if name in ("A0", "b0"):
        o = q // 6 if name == "A0" else q          # hidden unit of layer 1
        o2 = P1.index(o)                          # the layer-2 unit that reads it
        return {P2.index(o2)} if o2 in P2 else set()
    if name in ("A1", "b1"):
        o = q // W if name == "A1" else q
        return {P2.index(o)} if o in P2 else set()
    return {q // W if name == "A2" else q}


def test_parameter_layout_probe(orc):
    rng = np.random.default_rng(11)
    sh = orc.shape(6, 8, 2, 6)
    p, P1, P2 = selection_network(orc, rng)
    assert len(p) == orc.mlp_nparams(sh) == 182
    norm = np.concatenate([np.zeros(6), np.ones(6), np.zeros(6), np.ones(6)])
    z = np.ascontiguousarray(rng.uniform(-1.5, 1.5, (6, 4)))
    y0 = orc.mlp_apply(sh, p, norm, z, mode=0)
    for k in range(len(p)):
        q = p.copy()
        q[k] += np.float32(2.0 ** -5)
        y = orc.mlp_apply(sh, q, norm, z, mode=0)
        moved = {j for j in range(6) if np.any(y[j] != y0[j])}
        assert moved == reached_outputs(k, P1, P2), k


@pytest.mark.parametrize("width,hidden", [(64, 3), (16, 2), (5, 1), (4, 0)])
def test_numpy_network_agrees_with_c_oracle(orc, width, hidden):
    rng = np.random.default_rng(width + hidden)
    sh = orc.shape(6, width, hidden, 6)
    p = (orc.mlp_init(sh, 3) + 0.05 * rng.standard_normal(orc.mlp_nparams(sh))).astype(np.float32)
    zin = np.ascontiguousarray(rng.normal(size=(6, 300)) * np.array([1e-5, 1e-5, 1e-5, 1e-4, 1e-4, 1e-3])[:, None])
    zout = np.ascontiguousarray(zin * 1.7 + 0.1 * np.roll(zin, 1, axis=0))
    norm = orc.norm_stats(zin, zout, 300)
    net = me.unpack(p, width, hidden)
    y_c = orc.mlp_apply(sh, p, norm, zin, mode=0)
    y_n = me.forward(net, me.normalise_in(zin, norm))
    assert np.abs(me.normalise_out(y_c, norm) - y_n).max() < 1e-13
    idx = np.arange(0, 300, 2)
    loss_c, g_c = orc.mlp_loss_grad(sh, p, norm, zin, zout, idx, mode=0)
    loss_n, g_n = me.loss_grad(net, me.normalise_in(zin, norm)[idx], me.normalise_out(zout, norm)[idx])
    assert abs(loss_n / loss_c - 1) < 1e-13
    assert np.abs(g_n - g_c).max() <= 1e-12 * np.abs(g_c).max()


def bf16_like(orc):
    """The rounding points of an implementation whose hidden and output layers
    take bf16 weights and activations and whose first layer keeps 16
    significant bits of its operands, FP32 sums and output."""
    return me.Rounding(u_w=[2.0 ** -15, 2.0 ** -8, 2.0 ** -8, 2.0 ** -8],
                       u_x=[2.0 ** -15, 2.0 ** -8, 2.0 ** -8, 2.0 ** -8],
                       e_act=2.0 ** -20, u_acc=70 * 2.0 ** -24, u_out=2.0 ** -24, u_d=2.0 ** -8)


@pytest.fixture(scope="module")
def stage_pairs(orc):
    import workloads as W
    n = 2048
    wl = W.c3_stage(n=n, nsub=200)
    c = orc.fill_gaussian(n, 3, (0.0,) * 6, wl.bunch.sigma)
    r = orc.Ref.from_energy(wl.E_MeV)
    orc.push(c, wl.beamline[0], r)
    xin = c.copy()
    orc.push(c, [wl.beamline[1]], r)
    return xin, c, orc.norm_stats(xin, c, n)


def test_bound_zero_without_rounding(orc, stage_pairs):
    xin, _, norm = stage_pairs
    p = orc.mlp_init(orc.shape(), 5)
    rnd = me.Rounding(u_w=[0.0] * 4, u_x=[0.0] * 4)
    _, B, S = me.forward_bound(me.unpack(p, 64, 3), me.normalise_in(xin, norm), rnd)
    assert B.max() == 0.0 and S.max() == 0.0


def test_bound_covers_a_bf16_implementation(orc, stage_pairs):
    """The oracle's kernel-emulating mode is an actual implementation with
    those rounding points (bf16 weights and activations, split first layer):
    its distance from the FP64 network stays within the first-order bound and
    within a few probabilistic scales."""
    xin, _, norm = stage_pairs
    rng = np.random.default_rng(5)
    p = (orc.mlp_init(orc.shape(), 5) + 0.05 * rng.standard_normal(9158)).astype(np.float32)
    y, B, S = me.forward_bound(me.unpack(p, 64, 3), me.normalise_in(xin, norm), bf16_like(orc))
    y0 = orc.mlp_apply(orc.shape(), p, norm, xin, mode=0)
    y1 = orc.mlp_apply(orc.shape(), p, norm, xin, mode=1)
    d = np.abs(me.normalise_out(y1, norm) - me.normalise_out(y0, norm))
    assert np.all(d <= B)
    assert np.all(d <= 4.0 * S)
    assert np.median(d) > 1e-6          # the emulation does round: the check is not vacuous


def test_monte_carlo_spread_matches_probabilistic_scale(orc, stage_pairs):
    """Uniform perturbations of size u have standard deviation u/sqrt(3), so
    the ensemble's spread must be S/sqrt(3) to first order."""
    xin, _, norm = stage_pairs
    net = me.unpack(orc.mlp_init(orc.shape(), 7), 64, 3)
    x = me.normalise_in(xin[:, :256], norm)
    rnd = bf16_like(orc)
    Y = np.array([me.perturbed_forward(net, x, rnd, np.random.default_rng(k))[2] for k in range(48)])
    _, _, S = me.forward_bound(net, x, rnd)
    ratio = np.median(Y.std(axis=0, ddof=1) / (S / math.sqrt(3.0)))
    assert 0.9 < ratio < 1.1, ratio


def test_philox_known_answers(orc):
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(t, 16) for t in r]
        assert orc.philox(v[0:4], v[4:6]) == v[6:10]


def test_learning_rate_schedule(orc):
    """Half cosine from lr (first step) to lr_final (last step): endpoints,
    midpoint (lr + lr_final)/2, symmetry lr_t + lr_{T+1-t} = lr + lr_final,
    monotone decrease; constant when lr_final = lr."""
    T, a, b = 101, 1e-3, 1e-5
    lr = np.array([orc.lr_at(t, T, a, b) for t in range(1, T + 1)])
    assert lr[0] == a and abs(lr[-1] - b) < 1e-18
    assert abs(lr[50] - 0.5 * (a + b)) < 1e-18
    assert np.allclose(lr + lr[::-1], a + b, rtol=0, atol=1e-18)
    assert np.all(np.diff(lr) < 0)
    assert all(orc.lr_at(t, T, a, a) == a for t in (1, 50, 101))
    assert orc.lr_at(1, 1, a, b) == a
