"""GPU parity of the energy-dependent variants against the oracle: chromatic
quadrupoles and thin lenses (fused, unfused, inside stage and inference
kernels as transport gaps) and the stage with an energy-correlated gain.
1e-12 relative per coordinate, inputs from the oracle's fill."""
import numpy as np
import pytest

import workloads as W
from gpu_util import rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu
TOL = 1e-12


@pytest.fixture(scope="module")
def hbl():
    from paper_2402_17248_amd import hbl as h
    return h


def chromatic_lattice():
    """FODO cells with chromatic quads, a chromatic thin lens, a bend pair."""
    q = lambda k: W.Element(W.QUAD, L=0.5, k=k, chromatic=True)
    cell = [W.drift(0.2), q(+1.5), W.drift(0.4), q(-1.5), W.drift(0.2)]
    return cell * 3 + [W.Element(W.THIN_LENS, f=0.8, chromatic=True), W.sbend(0.5, 4e-3), W.drift(0.5),
                       W.sbend(0.5, -4e-3)]


def oracle_bunch(orc, n, seed):
    sig = (10e-6, 10e-6, 10e-6, 1e-4, 1e-4, 3e-3)        # wide energy spread: chromaticity matters
    return orc.fill_gaussian(n, seed, (0.0,) * 6, sig)


@pytest.mark.parametrize("n", [1, 63, 10_001])
def test_chromatic_lattice_fused_unfused_oracle(hbl, orc, n):
    els = chromatic_lattice()
    c = oracle_bunch(orc, n, 31)
    zf, zu = to_dev(c), to_dev(c)
    ref = hbl.Ref.from_energy(1000.0)
    lat = hbl.Lattice(els, ref)
    lat.push(zf, ref.copy(), fused=True, n=n)
    lat.push(zu, ref.copy(), fused=False, n=n)
    g, gu = to_host(zf, n), to_host(zu, n)
    assert np.array_equal(g, gu)
    achro = c.copy()
    orc.push(achro, [W.Element(e.kind, L=e.L, k=e.k, angle=e.angle, f=e.f) for e in els],
             orc.Ref.from_energy(1000.0))
    orc.push(c, els, orc.Ref.from_energy(1000.0))
    assert rel_err(g, c).max() < TOL
    if n > 1000:
        assert rel_err(achro, c).max() > 1e-4        # the chromatic terms are exercised


@pytest.mark.parametrize("n,nsub", [(2001, 300), (1, 200)])
def test_chirped_stage_with_chromatic_gaps(hbl, orc, n, nsub):
    """Chirped stage with chromatic triplets fused as its gaps, input recorded,
    against the oracle's lattice + stage + lattice."""
    wl = W.c3_chromatic(n=n, nsub=nsub)
    c = oracle_bunch(orc, n, 32)
    z = to_dev(c)
    rec = to_dev(np.zeros_like(c))
    ref = hbl.Ref.from_energy(wl.E_MeV)
    pre = hbl.Lattice(wl.beamline[0], ref)
    post_ref = ref.copy()
    post_ref.gamma += wl.beamline[1].dE_MeV / post_ref.mass_MeV
    post = hbl.Lattice(wl.beamline[2], post_ref)
    hbl.apply_stage(z, wl.beamline[1], ref, record=rec, n=n, pre=pre, post=post)
    g, r = to_host(z, n), to_host(rec, n)
    oref = orc.Ref.from_energy(wl.E_MeV)
    orc.push(c, wl.beamline[0], oref)
    assert rel_err(r, c).max() < TOL
    unchirped = c.copy()
    orc.push(unchirped, [W.Stage(L=0.3, n0_m3=1e23, dE_MeV=9000.0, nsub=nsub)], orc.Ref(gamma=oref.gamma, s=oref.s))
    orc.push(c, [wl.beamline[1]], oref)
    if n > 1:
        assert np.abs(unchirped[5] - c[5]).max() > 1e-6 * np.abs(c[5]).max()   # the chirp matters
    orc.push(c, wl.beamline[2], oref)
    assert rel_err(g, c).max() < TOL
    assert abs(ref.gamma / oref.gamma - 1) < 1e-15 and abs(ref.s - oref.s) < 1e-14


def test_chromatic_full_size_sampled(hbl, orc):
    """C3 chromatic variant at its size (1e6 particles, 2000 substeps), the
    launch shape of the benchmark study, sampled particles."""
    torch = __import__("torch")
    wl = W.c3_chromatic()
    n = wl.bunch.n
    z = hbl.new_bunch(n)
    hbl.fill_gaussian(z, wl.bunch.seed, (0.0,) * 6, wl.bunch.sigma, n=n)
    idx = np.sort(np.random.default_rng(4).choice(n, 2000, replace=False))
    idx[-1] = n - 1
    ti = torch.from_numpy(idx).cuda()
    c = orc.fill_gaussian(0, wl.bunch.seed, (0.0,) * 6, wl.bunch.sigma, idx=idx)
    z[:, ti] = torch.from_numpy(c).cuda()
    ref = hbl.Ref.from_energy(wl.E_MeV)
    for seg in wl.beamline:
        if isinstance(seg, list):
            hbl.Lattice(seg, ref).push(z, ref, n=n)
        else:
            hbl.apply_stage(z, seg, ref, n=n)
    torch.cuda.synchronize()
    g = np.ascontiguousarray(z[:, ti].cpu().numpy())
    orc.track(c, wl.beamline, orc.Ref.from_energy(wl.E_MeV))
    assert rel_err(g, c).max() < TOL


def test_surrogate_with_chromatic_gaps_bitwise(hbl, orc):
    """Inference with chromatic gaps fused equals chromatic lattice pushes
    around a plain inference call, bit for bit."""
    torch = __import__("torch")
    wl = W.c3_chromatic(n=10)
    n = 30_001
    c = oracle_bunch(orc, n, 33)
    sur = hbl.Surrogate(5)
    sig = (10e-6, 10e-6, 10e-6, 1e-4, 1e-4, 3e-3)
    sur.set_norm([0.0] * 6 + list(sig) + [0.0] * 6 + list(sig))
    ref = hbl.Ref.from_energy(wl.E_MeV)
    sur.set_stage(wl.beamline[1], ref)
    pre = hbl.Lattice(wl.beamline[0], ref)
    post_ref = ref.copy()
    post_ref.gamma += wl.beamline[1].dE_MeV / post_ref.mass_MeV
    post = hbl.Lattice(wl.beamline[2], post_ref)
    za, zb = to_dev(c), to_dev(c)
    ra = ref.copy()
    sur.apply(za, ra, n=n, pre=pre, post=post)
    rb = ref.copy()
    pre.push(zb, rb.copy(), n=n)
    sur.apply(zb, rb, n=n)
    post.push(zb, post_ref.copy(), n=n)
    torch.cuda.synchronize()
    assert torch.equal(za, zb)


def test_chirp_gain_factor_beyond_newton_range(hbl, orc):
    """Particles whose gain factor 1 + chirp t leaves [0, 2] take the kernel's
    division path (the Newton steps are sized for that range); both paths
    against the oracle."""
    n, chirp = 4001, 1e4
    c = oracle_bunch(orc, n, 34)
    c[2] = np.linspace(-1.05, 1.6, n) / chirp              # gain factor from -0.05 to 2.6
    st = W.Stage(L=0.3, n0_m3=1e23, dE_MeV=9000.0, nsub=400, chirp=chirp)
    z = to_dev(c)
    ref = hbl.Ref.from_energy(1000.0)
    hbl.apply_stage(z, st, ref, n=n)
    g = to_host(z, n)
    orc.push(c, [st], orc.Ref.from_energy(1000.0))
    assert np.all(np.isfinite(g))
    assert rel_err(g, c).max() < TOL
