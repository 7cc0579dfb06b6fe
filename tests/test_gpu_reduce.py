"""GPU parity of the diagnostics reductions (moments, emittances, paired
metrics) against the oracle's exact sums on the same bunch bytes."""
import math

import numpy as np
import pytest

import workloads as W
from gpu_util import to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hbl():
    from paper_2402_17248_amd import hbl as h
    return h


def moment_errors(orc, g_mean, g_cov, z):
    om, oc = orc.moments(z)
    C = orc.cov_matrix(oc)
    Cg = orc.cov_matrix(g_cov)
    sd = np.sqrt(np.diag(C))
    sd[sd == 0] = 1.0
    # a mean is compared on the scale max(|mean|, sigma): it is itself rounded
    em = np.abs((np.array(g_mean) - om) / np.maximum(sd, np.abs(om))).max()
    ec = np.abs((Cg - C) / np.outer(sd, sd)).max()
    return em, ec, oc


@pytest.mark.parametrize("n,offset", [(1, 0.0), (2, 0.0), (255, 0.0), (10_001, 0.0), (10_001, 1e4), (1_000_000, 0.0)])
def test_moments_parity(hbl, orc, n, offset):
    sig = np.array(W.BunchSpec(1, 1).sigma)
    mean = tuple(offset * sig)
    z = hbl.new_bunch(n)
    hbl.fill_gaussian(z, 11, mean, tuple(sig), n=n)
    g_mean, g_cov = hbl.moments(z, n=n)
    host = to_host(z, n)
    em, ec, oc = moment_errors(orc, g_mean, g_cov, host)
    assert em < 1e-13 and ec < 1e-13, (em, ec)
    # emittance within its conditioning of the exact one
    e_g = hbl.emittances(g_cov)
    e_o = orc.emittances(oc)
    C = orc.cov_matrix(oc)
    for p, (q, m) in enumerate(((0, 3), (1, 4), (2, 5))):
        if e_o[p] == 0:
            continue
        kappa = C[q, q] * C[m, m] / e_o[p] ** 2
        assert abs(e_g[p] / e_o[p] - 1) <= 4 * kappa * 1e-13 + 1e-15


def test_moments_of_correlated_stage_exit(hbl, orc):
    wl = W.c3_stage(n=50_001, nsub=500)
    n = wl.bunch.n
    z = hbl.new_bunch(n)
    hbl.fill_gaussian(z, 3, (0.0,) * 6, wl.bunch.sigma, n=n)
    ref = hbl.Ref.from_energy(wl.E_MeV)
    hbl.Lattice(wl.beamline[0], ref).push(z, ref, n=n)
    hbl.apply_stage(z, wl.beamline[1], ref, n=n)
    g_mean, g_cov = hbl.moments(z, n=n)
    em, ec, _ = moment_errors(orc, g_mean, g_cov, to_host(z, n))
    assert em < 1e-13 and ec < 1e-13


def test_moments_deterministic(hbl):
    n = 3_000_001
    z = hbl.new_bunch(n)
    hbl.fill_gaussian(z, 5, (0.0,) * 6, W.BunchSpec(1, 1).sigma, n=n)
    a = hbl.moments(z, n=n)
    b = hbl.moments(z, n=n)
    assert a == b


def test_nonfinite_detected(hbl):
    n = 1000
    z = hbl.new_bunch(n)
    hbl.fill_gaussian(z, 5, (0.0,) * 6, W.BunchSpec(1, 1).sigma, n=n)
    z[3, 500] = float("nan")
    with pytest.raises(hbl.HblError) as ei:
        hbl.moments(z, n=n)
    assert ei.value.status == hbl.HBL_ENONFINITE


def test_compare_parity(hbl, orc):
    n = 20_001
    sig = W.BunchSpec(1, 1).sigma
    f = hbl.new_bunch(n)
    hbl.fill_gaussian(f, 8, (0.0,) * 6, sig, n=n)
    s = f.clone()
    s[:, :n] = s[:, :n] * 1.001 + 1e-9
    r, c, e = hbl.compare(s, f, n=n)
    ro, co, eo = orc.compare(to_host(s, n), to_host(f, n))
    assert np.abs(np.array(r) - ro).max() < 1e-12 * np.abs(ro).max()
    assert np.abs(np.array(c) - co).max() < 1e-12 + 1e-10 * np.abs(co).max()
    assert np.abs(np.array(e) - eo).max() < 1e-10


def test_moments_async_matches_sync(hbl):
    torch = __import__("torch")
    n = 100_000
    z = hbl.new_bunch(n)
    hbl.fill_gaussian(z, 5, (0.0,) * 6, W.BunchSpec(1, 1).sigma, n=n)
    out = torch.empty(27, dtype=torch.float64, device="cuda")
    hbl.moments_async(z, out, n=n)
    m, c = hbl.moments(z, n=n)
    torch.cuda.synchronize()
    assert out.cpu().tolist() == m + c
