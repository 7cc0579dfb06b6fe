"""GPU parity of the paper-shaped PReLU surrogate (§3 Eq. 2 and 3; 3 x 700
and 5 x 900 hidden layers) against the oracle's bf16-emulation mode, through
the C ABI.

Expected differences: the oracle sums each pre-activation in FP64 and rounds
once; the GPU sums bf16 products in FP32 on the matrix cores (relative
rounding ~K 2^-24 of the partial sums, K <= 960) and forms the first layer
with FP32 fused multiply-adds.  A pre-activation within that distance of a
bf16 rounding boundary rounds the other way: a one-ulp (2^-8 relative)
change of that activation, in a small fraction of the activations; PReLU is
piecewise linear, so such a change reaches the output scaled by the weights
(~1/sqrt(W)) without amplification.  With ~1e-3 of the activations flipped
(FP32 sums of up to 960 terms are good to ~sqrt(K) 2^-24 ~ 2e-6 relative,
against a bf16 half-ulp of 2e-3) a 5 x 900 network flips a few activations
per particle, each moving an output by ~2^-8 x 1/sqrt(W) ~ 1e-4 (normalised
units): the median output agrees to rounding, a few percent of the
particles move by ~1e-4, and nothing moves by much more than 1e-3."""
import numpy as np
import pytest

import workloads as W
from gpu_util import to_dev, to_host

pytestmark = pytest.mark.gpu

SHAPES = [(700, 3), (900, 5)]


@pytest.fixture(scope="module")
def hbl():
    from paper_2402_17248_amd import hbl as h
    return h


def norm_for(sigma):
    sd = np.asarray(sigma, dtype=float)
    return np.concatenate([0.01 * sd, sd, 0.3 * sd, 1.7 * sd])


def bunch(orc, n, seed):
    sigma = W.c3_stage(n=8).bunch.sigma
    return orc.fill_gaussian(n, seed, (0.0,) * 6, sigma), norm_for(sigma)


def perturbed(orc, sh, seed):
    p = orc.prelu_init(sh, seed)
    rng = np.random.default_rng(seed)
    q = (p + 0.02 * rng.standard_normal(p.shape)).astype(np.float32)
    return q


def compare(g, c, norm):
    d = np.abs(g - c) / norm[18:24, None]
    return d.max(), np.median(d), np.mean(d.max(axis=0) > 1e-3)


@pytest.mark.parametrize("width,hidden", [(700, 3), (900, 5), (64, 1), (100, 2)])
def test_init_matches_oracle(hbl, orc, width, hidden):
    for seed in (0, 2**40 + 3):
        net = hbl.PreluNet(width, hidden, seed)
        assert np.array_equal(net.get_params(), orc.prelu_init(orc.shape(width=width, hidden=hidden), seed))


@pytest.mark.parametrize("width,hidden", SHAPES)
def test_forward_parity_paper_shapes(hbl, orc, width, hidden):
    sh = orc.shape(width=width, hidden=hidden)
    m = 1000                                   # 4 tiles of 256, the last ragged
    x, norm = bunch(orc, m, 21)
    p = perturbed(orc, sh, 7)
    net = hbl.PreluNet(width, hidden, 0)
    net.set_params(p)
    net.set_norm(norm)
    z = to_dev(x)
    net.apply(z, n=m)
    g = to_host(z, m)
    c = orc.prelu_apply(sh, p, norm, x, mode=1)
    mx, med, frac = compare(g, c, norm)
    print(f"{width}x{hidden}: max {mx:.3e} median {med:.3e} frac>1e-3 {frac:.4f}")
    assert mx < 5e-3 and med < 1e-7 and frac < 0.01


@pytest.mark.parametrize("width,m", [(100, 1), (100, 255), (100, 256), (100, 257), (100, 65536 + 300),
                                     (520, 1), (520, 257), (520, 65536 + 300)])
def test_forward_ragged_and_chunked(hbl, orc, width, m):
    """Ragged tiles and several chunks, on row-major activations (W' = 128)
    and on K-blocked ones (W' = 576), where a chunk's rows set the stride of
    the blocks."""
    sh = orc.shape(width=width, hidden=2)
    x, norm = bunch(orc, m + 5, 22)
    p = perturbed(orc, sh, 8)
    net = hbl.PreluNet(width, 2, 0)
    net.set_chunk(65536)                               # m = 65536 + 300 spans two chunks
    net.set_params(p)
    net.set_norm(norm)
    z = to_dev(x)
    net.apply(z, n=m)
    g = to_host(z, m + 5)
    c = orc.prelu_apply(sh, p, norm, np.ascontiguousarray(x[:, :m]), mode=1)
    mx, med, frac = compare(g[:, :m], c, norm)
    print(f"m={m}: max {mx:.3e} median {med:.3e}")
    assert mx < 5e-3 and med < 1e-7
    assert np.array_equal(g[:, m:], x[:, m:])          # particles past n untouched


@pytest.mark.parametrize("width", [128, 520])
def test_gaps_equal_separate_calls(hbl, orc, width):
    """pre lattice, network, post lattice in the same launches == three calls
    (bitwise), on row-major and on K-blocked activations."""
    m = 3000
    wl = W.c3_chromatic(n=8)
    x, norm = bunch(orc, m, 23)
    net = hbl.PreluNet(width, 2, 3)
    net.set_norm(norm)
    stage = wl.beamline[1]
    for chromatic in (False, True):
        trip = W.triplet(chromatic=chromatic)
        ref0 = hbl.Ref.from_energy(wl.E_MeV)
        net.set_stage(stage, ref0)
        pre = hbl.Lattice(trip, ref0)
        ref_exit = ref0.copy()
        ref_exit.gamma += stage.dE_MeV / ref_exit.mass_MeV
        post = hbl.Lattice(trip, ref_exit)
        z1 = to_dev(x)
        r1 = ref0.copy()
        net.apply(z1, r1, n=m, pre=pre, post=post)
        z2 = to_dev(x)
        r2 = ref0.copy()
        pre.push(z2, r2, n=m)
        net.apply(z2, r2, n=m)
        post.push(z2, r2, n=m)
        assert np.array_equal(to_host(z1, m), to_host(z2, m)), chromatic
        assert r1.gamma == r2.gamma


@pytest.mark.parametrize("width,hidden", SHAPES)
def test_full_size_sampled(hbl, orc, width, hidden):
    """The C4 inference workload (1e7 particles) at the paper's shapes; 300
    sampled particles against the oracle, which fills the same particles."""
    sh = orc.shape(width=width, hidden=hidden)
    sigma = W.c3_stage(n=8).bunch.sigma
    norm = norm_for(sigma)
    p = perturbed(orc, sh, 9)
    net = hbl.PreluNet(width, hidden, 0)
    net.set_params(p)
    net.set_norm(norm)
    N = W.C4_INFER_N
    z = hbl.new_bunch(N)
    hbl.fill_gaussian(z, W.C4_INFER_SEED, (0.0,) * 6, sigma, n=N)
    torch = __import__("torch")
    idx = np.sort(np.random.default_rng(4).choice(N, 300, replace=False))
    idx[-1] = N - 1
    x0 = orc.fill_gaussian(0, W.C4_INFER_SEED, (0.0,) * 6, sigma, idx=idx)
    net.apply(z, n=N)
    g = np.ascontiguousarray(z[:, torch.from_numpy(idx).cuda()].cpu().numpy())
    c = orc.prelu_apply(sh, p, norm, x0, mode=1)
    mx, med, frac = compare(g, c, norm)
    print(f"full {width}x{hidden}: max {mx:.3e} median {med:.3e} frac>1e-3 {frac:.4f}")
    assert mx < 5e-3 and med < 1e-7 and frac < 0.01


@pytest.mark.parametrize("width,hidden", [(8, 1), (72, 2), (136, 3), (250, 2), (500, 2), (520, 7), (600, 2),
                                          (750, 2), (800, 2), (880, 2), (1024, 2)])
def test_forward_parity_other_widths(hbl, orc, width, hidden):
    """Widths that pick every kind of M block (4 to 12 MFMA tiles, one to
    eight blocks per layer, row-major), every K-blocked width class (W' =
    512 .. 896: 8 to 14 row tiles per M block, persistent up to 13), the
    deepest and the widest network allowed."""
    sh = orc.shape(width=width, hidden=hidden)
    m = 700
    x, norm = bunch(orc, m, 24)
    p = perturbed(orc, sh, 10)
    net = hbl.PreluNet(width, hidden, 0)
    net.set_params(p)
    net.set_norm(norm)
    z = to_dev(x)
    net.apply(z, n=m)
    g = to_host(z, m)
    c = orc.prelu_apply(sh, p, norm, x, mode=1)
    mx, med, frac = compare(g, c, norm)
    print(f"{width}x{hidden}: max {mx:.3e} median {med:.3e}")
    assert mx < 5e-3 and med < 1e-7 and frac < 0.01


@pytest.mark.parametrize("width", [136, 600])
def test_chunk_size_does_not_change_results(hbl, orc, width):
    """Chunking only splits the particles: any chunk gives the same bits, on
    row-major activations and on K-blocked ones (whose block stride is the
    chunk's row count)."""
    m = 5000
    x, norm = bunch(orc, m, 25)
    net = hbl.PreluNet(width, 3, 7)
    net.set_norm(norm)
    outs = []
    for ch in (65536, 256, 1024, 98304):
        net.set_chunk(ch)
        z = to_dev(x)
        net.apply(z, n=m)
        outs.append(to_host(z, m))
    assert all(np.array_equal(outs[0], o) for o in outs[1:])
    with pytest.raises(hbl.HblError):
        net.set_chunk(1000)
