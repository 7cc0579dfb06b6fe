"""GPU parity of the surrogate network (§3 Eq. 3-4, Adam) through the C ABI,
against the FP64 network of the CPU oracle.

Reference: the oracle's FP64 evaluation (mode 0), the network as defined.
Allowance: what the library's documented rounding points allow
(tests/rounding_contract.py; oracle/mlp_error.py derives it):

* forward, per output and particle: within the first-order worst-case bound B
  and within LAM = 7 probabilistic scales S (independent rounding errors,
  Hoeffding: each output exceeds 7 S with probability <= 5e-11), and the
  median distance below one S;
* gradient, per parameter: within 8 standard deviations of a 64-member
  Monte-Carlo-arithmetic ensemble of the FP64 gradient with those rounding
  points randomised (plus the FP32 rounding of the returned value), and per
  tensor a relative Frobenius distance below 3 x the ensemble's.

A secondary check per test compares with the oracle's kernel-emulating mode
(mode 1), which follows the kernel's own rounding (its tanh scale fold and
first-layer split) with FP64 sums and an exact tanh: there the two agree to
~1e-6 except where a value within ~1e-7 of a bf16 rounding boundary rounds
the other way on one side."""
import os
import tempfile

import numpy as np
import pytest

import workloads as W
from gpu_util import to_dev, to_host
from oracle import mlp_error as me
from rounding_contract import LAM, SURROGATE

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hbl():
    from paper_2402_17248_amd import hbl as h
    return h


@pytest.fixture(scope="module")
def pairs(hbl, orc):
    """2^14 stage pairs made by the oracle (triplet, then the fine-step stage,
    its input kept) and uploaded: (n, inputs on device, outputs on device,
    inputs on host, outputs on host, stage, reference at the stage entrance)."""
    n = 1 << 14
    wl = W.c3_stage(n=n, nsub=400)
    c = orc.fill_gaussian(n, 3, (0.0,) * 6, wl.bunch.sigma)
    oref = orc.Ref.from_energy(wl.E_MeV)
    orc.push(c, wl.beamline[0], oref)
    xin = c.copy()
    orc.push(c, [wl.beamline[1]], oref)
    entry = hbl.Ref.from_energy(wl.E_MeV)
    entry.s = oref.s - wl.beamline[1].L
    return n, to_dev(xin), to_dev(c), xin, c, wl.beamline[1], entry


def perturbed(orc, seed):
    p = orc.mlp_init(orc.shape(), seed)
    rng = np.random.default_rng(seed)
    return (p + 0.05 * rng.standard_normal(p.shape)).astype(np.float32)


def check_forward(g, xin, p, norm, what):
    """g: GPU output bunch (6, m) for raw inputs xin (6, m).  Returns the
    normalised distance from the FP64 network and the scales, after checking
    the bound and the probabilistic scale."""
    net = me.unpack(p, 64, 3)
    y, B, S = me.forward_bound(net, me.normalise_in(xin, norm), SURROGATE)
    d = np.abs(me.normalise_out(g, norm) - y)
    r = d / S
    print(f"{what}: |gpu - fp64| max {d.max():.3e} median {np.median(d):.3e}; bound B median "
          f"{np.median(B):.3e}, max d/B {np.max(d / B):.3f}; d/S max {r.max():.2f} median {np.median(r):.3f}",
          flush=True)
    assert np.all(d <= B), np.max(d / B)
    assert np.all(r <= LAM), r.max()
    assert np.median(r) < 1.0, np.median(r)
    return d


def test_init_matches_oracle(hbl, orc):
    for seed in (0, 101, 2**40 + 3):
        s = hbl.Surrogate(seed)
        assert np.array_equal(s.get_params(), orc.mlp_init(orc.shape(), seed))


def test_forward_parity(hbl, orc, pairs):
    n, rec, out, xin, xout, _, _ = pairs
    norm = orc.norm_stats(xin, xout, n)
    s = hbl.Surrogate(0)
    p = perturbed(orc, 5)
    s.set_params(p)
    s.set_norm(norm)
    m = 10_001
    z = rec[:, :m + 1].clone()
    s.apply(z, n=m)
    g = to_host(z, m)
    x = np.ascontiguousarray(xin[:, :m])
    check_forward(g, x, p, norm, "forward 10001")
    # secondary: the kernel-emulating mode (same rounding points, FP64 sums, exact tanh)
    c = orc.mlp_apply(orc.shape(), p, norm, x, mode=1)
    d1 = np.abs(g - c) / norm[18:24, None]
    frac = np.mean(d1.max(axis=0) > 1e-4)
    print(f"vs kernel emulation: median {np.median(d1):.2e} max {d1.max():.2e}, particles beyond 1e-4 {frac:.4f}",
          flush=True)
    assert np.median(d1) < 1e-6
    assert d1.max() < 1e-2
    assert frac < 0.01


@pytest.mark.parametrize("m", [1, 63, 64, 65, 130])
def test_forward_ragged_sizes(hbl, orc, pairs, m):
    n, rec, out, xin, xout, _, _ = pairs
    norm = orc.norm_stats(xin, xout, n)
    s = hbl.Surrogate(0)
    p = perturbed(orc, 6)
    s.set_params(p)
    s.set_norm(norm)
    z = rec.clone()
    s.apply(z, n=m)
    g = to_host(z, n)
    net = me.unpack(p, 64, 3)
    y, B, S = me.forward_bound(net, me.normalise_in(np.ascontiguousarray(xin[:, :m]), norm), SURROGATE)
    d = np.abs(me.normalise_out(np.ascontiguousarray(g[:, :m]), norm) - y)
    assert np.all(d <= B) and np.all(d <= LAM * S)
    assert np.array_equal(g[:, m:], xin[:, m:])          # particles past n untouched


def test_forward_full_size_sampled(hbl, orc, pairs):
    n, rec, out, xin, xout, _, _ = pairs
    norm = orc.norm_stats(xin, xout, n)
    s = hbl.Surrogate(0)
    p = perturbed(orc, 7)
    s.set_params(p)
    s.set_norm(norm)
    N = W.C4_INFER_N
    z = hbl.new_bunch(N)
    mean, sd = tuple(norm[0:6]), tuple(norm[6:12])
    hbl.fill_gaussian(z, W.C4_INFER_SEED, mean, sd, n=N)
    torch = __import__("torch")
    idx = np.sort(np.random.default_rng(3).choice(N, 2000, replace=False))
    idx[-1] = N - 1
    ti = torch.from_numpy(idx).cuda()
    x0 = orc.fill_gaussian(0, W.C4_INFER_SEED, mean, sd, idx=idx)   # same particles, the oracle's fill
    s.apply(z, n=N)
    g = np.ascontiguousarray(z[:, ti].cpu().numpy())
    check_forward(g, x0, p, norm, "forward 1e7 sampled")


TENSORS = [("W0", 0, 384), ("b0", 384, 448), ("W1", 448, 4544), ("b1", 4544, 4608), ("W2", 4608, 8704),
           ("b2", 8704, 8768), ("W3", 8768, 9152), ("b3", 9152, 9158)]


def rel_fro(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)


def mca_gradient(p, norm, xin, xout, idx, K=64):
    """FP64 loss and gradient of the batch idx, and the spread of K
    Monte-Carlo-arithmetic passes with the documented rounding points."""
    net = me.unpack(p, 64, 3)
    x = me.normalise_in(np.ascontiguousarray(xin[:, idx]), norm)
    yt = me.normalise_out(np.ascontiguousarray(xout[:, idx]), norm)
    loss, g = me.loss_grad(net, x, yt)
    draws = [me.loss_grad(net, x, yt, SURROGATE, np.random.default_rng(7000 + k)) for k in range(K)]
    Ls = np.array([d[0] for d in draws])
    G = np.array([d[1] for d in draws])
    return loss, g, Ls.std(ddof=1), G.std(axis=0, ddof=1)


def check_gradient(gg, g64, sig, what):
    d = np.abs(gg.astype(np.float64) - g64)
    allow = 8.0 * sig + 2.0 * 2.0 ** -24 * np.abs(g64) + 1e-12 * np.abs(g64).max()
    print(f"{what}: max |dg|/sigma {np.max(d / np.maximum(sig, 1e-300)):.2f}, median "
          f"{np.median(d / np.maximum(sig, 1e-300)):.2f}", flush=True)
    assert np.all(d <= allow), np.argmax(d / allow)
    for name, a, b in TENSORS:
        rf = rel_fro(gg[a:b].astype(np.float64), g64[a:b])
        spread = np.linalg.norm(sig[a:b]) / np.linalg.norm(g64[a:b])
        assert rf < 3.0 * spread + 1e-6, (name, rf, spread)


def test_gradient_parity(hbl, orc, pairs):
    n, rec, out, xin, xout, _, _ = pairs
    norm = orc.norm_stats(xin, xout, n)
    s = hbl.Surrogate(0)
    p = perturbed(orc, 8)
    s.set_params(p)
    s.set_norm(norm)
    idx = np.random.default_rng(4).choice(n, 512, replace=False).astype(np.int32)
    loss_g, g = s.loss_grad(rec, out, idx)
    loss64, g64, sig_l, sig = mca_gradient(p, norm, xin, xout, idx)
    print(f"loss gpu {loss_g:.8e} fp64 {loss64:.8e} (|d|/sigma {abs(loss_g - loss64) / sig_l:.2f})", flush=True)
    assert abs(loss_g - loss64) <= 8.0 * sig_l + 1e-7 * loss64
    check_gradient(g, g64, sig, "gradient 512")
    # secondary: the kernel-emulating mode
    _, go = orc.mlp_loss_grad(orc.shape(), p, norm, xin, xout, idx.astype(np.int64), mode=1)
    worst = max(rel_fro(g[a:b].astype(np.float64), go[a:b]) for _, a, b in TENSORS)
    print(f"vs kernel emulation: worst per-tensor relative Frobenius {worst:.2e}", flush=True)
    assert worst < 1e-3


def test_first_adam_step_and_epoch_order(hbl, orc, pairs):
    """One optimizer step of training equals the oracle's Adam applied to the
    FP64 gradient of the first batch of the oracle's epoch-0 Fisher-Yates
    order.  Adam's first step moves a parameter by lr g/(|g| + eps) ~ lr
    sign(g): it must agree wherever the FP64 gradient is farther from zero
    than the rounding can move it (8 ensemble deviations); elsewhere the
    sign may differ and the step by at most 2 lr."""
    n, rec, out, xin, xout, _, _ = pairs
    s = hbl.Surrogate(11)
    p0 = orc.mlp_init(orc.shape(), 11)
    assert np.array_equal(s.get_params(), p0.astype(np.float32))
    s.train(rec, out, n, batch=64, epochs=1, lr=1e-3, train_frac=0.7, shuffle_seed=77, max_steps=1)
    p1 = s.get_params().astype(np.float64)
    ntr = int(round(0.7 * n))
    on = orc.norm_stats(xin, xout, ntr)
    assert np.allclose(s.get_norm(), on, rtol=1e-13, atol=0)
    first = orc.epoch_perm(ntr, 77, 0)[:64]
    _, g64, _, sig = mca_gradient(p0, on, xin, xout, first)
    want, _, _ = orc.adam_step(p0, np.zeros(len(p0)), np.zeros(len(p0)), g64, 1, lr=1e-3)
    d = np.abs(p1 - want)
    firm = np.abs(g64) > 8.0 * sig + 1e-6 * np.abs(g64).max()
    print(f"first Adam step: {firm.mean():.3f} of the parameters have a firm gradient sign; "
          f"max step difference there {d[firm].max():.2e}", flush=True)
    assert firm.mean() > 0.5
    assert np.all(d[firm] <= 1e-6)
    assert d.max() <= 2e-3 + 1e-6


def test_training_curve_matches_oracle(hbl, orc, pairs):
    """Three epochs of the same recipe (same epoch orders and rates) on the
    GPU and in the oracle's FP64 training: the per-epoch training and test
    losses agree to 10 % (the two runs take different rounding at every step,
    and Adam's normalised steps let small gradient differences move the
    parameters by up to lr each)."""
    n, rec, out, xin, xout, _, _ = pairs
    s = hbl.Surrogate(12)
    p0 = orc.mlp_init(orc.shape(), 12)
    assert np.array_equal(s.get_params(), p0.astype(np.float32))
    log = s.train(rec, out, n, batch=256, epochs=3, lr=3e-3, lr_final=3e-4, shuffle_seed=5)
    _, _, olog = orc.mlp_train(orc.shape(), p0, xin, xout, batch=256, epochs=3, lr=3e-3, lr_final=3e-4,
                               shuffle_seed=5, mode=0)
    print("loss log gpu", log.tolist(), "oracle fp64", olog.tolist(), flush=True)
    assert np.all(np.isfinite(log))
    assert log[-1, 1] < 0.7 * log[0, 1]
    assert np.all(np.abs(log / olog - 1) < 0.1), (log, olog)


def test_save_load_roundtrip(hbl, orc, pairs):
    n, rec, out, xin, xout, stage, entry = pairs
    s = hbl.Surrogate(3)
    s.train(rec, out, n, batch=256, epochs=1, lr=1e-3, shuffle_seed=1)
    s.set_stage(stage, entry)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "m.hbls")
        s.save(path)
        t = hbl.Surrogate.load(path)
        assert np.array_equal(s.get_params(), t.get_params())
        assert s.get_norm() == t.get_norm()
        z1, z2 = rec.clone(), rec.clone()
        r1, r2 = entry.copy(), entry.copy()
        s.apply(z1, r1, n=n)
        t.apply(z2, r2, n=n)
        __import__("torch").cuda.synchronize()
        assert __import__("torch").equal(z1, z2)
        assert (r1.gamma, r1.s) == (r2.gamma, r2.s)
        with open(path, "r+b") as fh:
            fh.seek(200)
            b = fh.read(1)
            fh.seek(200)
            fh.write(bytes([b[0] ^ 1]))
        with pytest.raises(hbl.HblError) as ei:
            hbl.Surrogate.load(path)
        assert ei.value.status == hbl.HBL_EIO


def test_apply_moves_reference_and_checks_entry(hbl, orc, pairs):
    n, rec, out, xin, xout, stage, entry = pairs
    s = hbl.Surrogate(0)
    s.set_norm(orc.norm_stats(xin, xout, n))
    s.set_stage(stage, entry)
    r = entry.copy()
    s.apply(rec.clone(), r, n=n)
    assert abs(r.gamma - (entry.gamma + stage.dE_MeV / hbl.MEC2_MEV)) < 1e-9 and abs(r.s - entry.s - stage.L) < 1e-15
    bad = hbl.Ref.from_energy(2000.0)
    with pytest.raises(hbl.HblError) as ei:
        s.apply(rec.clone(), bad, n=n)
    assert ei.value.status == hbl.HBL_EINVAL


def test_keep_best_restores_lowest_test_loss_epoch(hbl, orc, pairs):
    """keep_best ends with the parameters after the epoch of lowest test loss:
    with a constant learning rate (the schedule then does not depend on the
    epoch count) and deterministic training, they equal bit for bit those of
    a second run from the same start stopped right after that epoch, and a
    run without keep_best ends with the last epoch's parameters."""
    n, rec, out, _, _, _, _ = pairs
    cfg = dict(batch=256, epochs=10, lr=5e-3, shuffle_seed=9)
    a = hbl.Surrogate(21)
    log = a.train(rec, out, n, keep_best=True, **cfg)
    best = int(np.argmin(log[:, 1]))
    print(f"keep_best: test losses {log[:, 1].tolist()}, lowest after epoch {best}", flush=True)
    b = hbl.Surrogate(21)
    log_b = b.train(rec, out, n, **{**cfg, "epochs": best + 1})
    assert np.array_equal(log_b, log[: best + 1])
    assert np.array_equal(a.get_params(), b.get_params())
    c = hbl.Surrogate(21)
    log_c = c.train(rec, out, n, **cfg)
    assert np.array_equal(log_c, log)
    if best < cfg["epochs"] - 1:
        assert not np.array_equal(c.get_params(), a.get_params())


def test_keep_best_by_test_split_emittance(hbl, orc, pairs):
    """keep_best=2 ends with the parameters, among the epochs of the last
    quarter whose test loss is within 10 % of those epochs' lowest, whose
    predicted test outputs have the emittances of (x, px) and (y, py) closest
    to the true test outputs'.  With a constant rate the candidates are the
    parameters of runs stopped after each of those epochs: the kept
    parameters equal, bit for bit, those of the eligible candidate with the
    lowest max_p |eps_pred,p / eps_true,p - 1| on the test split (computed
    here through hbl_compare)."""
    import torch
    n, rec, out, _, _, stage, entry = pairs
    cfg = dict(batch=256, epochs=16, lr=5e-3, shuffle_seed=13)
    ntr = int(round(0.7 * n))
    nte = n - ntr
    tin, tout = hbl.new_bunch(nte), hbl.new_bunch(nte)
    tin[:, :nte] = rec[:, ntr:n]
    tout[:, :nte] = out[:, ntr:n]
    a = hbl.Surrogate(31)
    log = a.train(rec, out, n, keep_best=2, **cfg)
    first = cfg["epochs"] - cfg["epochs"] // 4
    losses = log[first:, 1].astype(np.float64)
    scores, params = [], []
    for ep in range(first, cfg["epochs"]):
        b = hbl.Surrogate(31)
        b.train(rec, out, n, **{**cfg, "epochs": ep + 1})
        b.set_stage(stage, entry)
        zs = tin.clone()
        b.apply(zs, entry.copy(), n=nte)
        torch.cuda.synchronize()
        _, _, e = hbl.compare(zs, tout, n=nte)
        scores.append(max(abs(e[0]), abs(e[1])))
        params.append(b.get_params())
    ok = losses <= 1.1 * losses.min()
    cand = np.where(ok, scores, np.inf)
    k = int(np.argmin(cand))
    print(f"keep_best=2: last-quarter test losses {losses.tolist()}, emittance scores {scores}; kept {k}",
          flush=True)
    srt = sorted(cand)
    assert len(srt) < 2 or not np.isfinite(srt[1]) or srt[1] - srt[0] > 1e-12 * srt[1]   # a clear winner
    assert np.array_equal(a.get_params(), params[k])


def test_resume_after_save_and_load(hbl, orc, pairs):
    """Checkpoint and resume: 2 epochs, save, load into a new handle, resume
    for 3 more equals one run of 5 epochs bit for bit (constant rate: the
    schedule then does not depend on the call; same pairs and recipe), the
    resumed call's losses equal the single run's epochs 2-4, and a resume
    that cannot continue (no model, or a step count that is not a whole
    number of epochs) is rejected before anything runs."""
    n, rec, out, _, _, stage, entry = pairs
    cfg = dict(batch=256, lr=2e-3, shuffle_seed=3)
    a = hbl.Surrogate(41)
    log_a = a.train(rec, out, n, epochs=2, **cfg)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "ckpt.hbls")
        a.save(path)
        b = hbl.Surrogate.load(path)
    log_b = b.train(rec, out, n, epochs=3, resume=True, **cfg)
    c = hbl.Surrogate(41)
    log_c = c.train(rec, out, n, epochs=5, **cfg)
    print(f"resume: single-run test losses {log_c[:, 1].tolist()}, 2 + 3 resumed {log_a[:, 1].tolist()} "
          f"{log_b[:, 1].tolist()}", flush=True)
    assert np.array_equal(log_a, log_c[:2]) and np.array_equal(log_b, log_c[2:])
    assert np.array_equal(b.get_params(), c.get_params())
    with pytest.raises(hbl.HblError) as ei:
        hbl.Surrogate(42).train(rec, out, n, epochs=1, resume=True, **cfg)
    assert ei.value.status == hbl.HBL_EINVAL
    e = hbl.Surrogate(43)
    e.train(rec, out, n, epochs=1, max_steps=5, **cfg)
    with pytest.raises(hbl.HblError) as ei:
        e.train(rec, out, n, epochs=1, resume=True, **cfg)
    assert ei.value.status == hbl.HBL_EINVAL and "whole number of epochs" in str(ei.value)


def test_concurrent_training_equals_sequential(hbl, pairs):
    """Several trainings at once, each on a stream and host thread of its own
    (train_concurrently, as the staged chain trains its stages), give the
    networks, normalisations and loss curves of one-after-another training
    bitwise, for each model-selection mode."""
    from paper_2402_17248_amd.chain import train_concurrently
    n, rec, out, _, _, _, _ = pairs
    kws = [dict(batch=512, epochs=4, lr=1e-3, lr_final=1e-4, train_frac=0.7, shuffle_seed=10 + j, keep_best=kb)
           for j, kb in enumerate((0, 1, 2))]
    seq = []
    for j, kw in enumerate(kws):
        s = hbl.Surrogate(20 + j)
        curve = s.train(rec, out, n, **kw)
        seq.append((s.get_params(), s.get_norm(), curve))
    nets = [hbl.Surrogate(20 + j) for j in range(len(kws))]
    curves = train_concurrently([(nets[j], rec, out, n, kws[j]) for j in range(len(kws))])
    for j in range(len(kws)):
        assert np.array_equal(nets[j].get_params(), seq[j][0]), j
        assert np.array_equal(np.asarray(nets[j].get_norm()), np.asarray(seq[j][1])), j
        assert np.array_equal(curves[j], seq[j][2]), j
