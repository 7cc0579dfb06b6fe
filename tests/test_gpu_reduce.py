"""GPU parity of the diagnostics reductions (moments, emittances, paired
metrics) against the oracle's exact sums on the same bunch bytes (bunches
made by the oracle and uploaded)."""
import math

import numpy as np
import pytest

import workloads as W
from gpu_util import to_dev

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
    host = orc.fill_gaussian(n, 11, mean, tuple(sig))
    z = to_dev(host)
    g_mean, g_cov = hbl.moments(z, n=n)
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
    host = orc.fill_gaussian(n, 3, (0.0,) * 6, wl.bunch.sigma)
    orc.track(host, wl.beamline[:2], orc.Ref.from_energy(wl.E_MeV))
    g_mean, g_cov = hbl.moments(to_dev(host), n=n)
    em, ec, _ = moment_errors(orc, g_mean, g_cov, host)
    assert em < 1e-13 and ec < 1e-13


def test_moments_full_size_tiled(hbl, orc):
    """At the benchmark size (2.5e7, the launch shape the chain step uses):
    a bunch made of 25 copies of a 1e6-particle oracle bunch has that bunch's
    mean and covariance."""
    torch = __import__("torch")
    m, reps = 1_000_000, 25
    host = orc.fill_gaussian(m, 21, (0.0,) * 6, W.BunchSpec(1, 1).sigma)
    orc.track(host, [W.triplet()], orc.Ref.from_energy(1000.0))
    z = torch.from_numpy(host).cuda().repeat(1, reps).contiguous()
    g_mean, g_cov = hbl.moments(z, n=m * reps)
    em, ec, _ = moment_errors(orc, g_mean, g_cov, host)
    assert em < 1e-13 and ec < 1e-13, (em, ec)
    out = torch.empty(27, dtype=torch.float64, device="cuda")
    hbl.moments_async(z, out, n=m * reps)
    torch.cuda.synchronize()
    assert out.cpu().tolist() == g_mean + g_cov


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
    fh = orc.fill_gaussian(n, 8, (0.0,) * 6, sig)
    sh = fh * 1.001 + 1e-9
    r, c, e = hbl.compare(to_dev(sh), to_dev(fh), n=n)
    ro, co, eo = orc.compare(sh, fh)
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


def test_reductions_on_two_streams_do_not_share_a_workspace(hbl):
    """Reductions enqueued on different streams at the same time (each stream
    has a workspace of its own) give exactly the results of one-at-a-time
    reductions: asynchronous moments of two bunches on two streams, repeated
    so that the launches overlap, and synchronous moments from two host
    threads."""
    import threading
    torch = __import__("torch")
    n = 4_000_001
    sig = W.BunchSpec(1, 1).sigma
    za, zb = hbl.new_bunch(n), hbl.new_bunch(n)
    hbl.fill_gaussian(za, 11, (0.0,) * 6, sig, n=n)
    hbl.fill_gaussian(zb, 12, (1e-6,) * 6, sig, n=n)
    want_a, want_b = hbl.moments(za, n=n), hbl.moments(zb, n=n)
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    for st in (sa, sb):
        st.wait_stream(torch.cuda.current_stream())
    outs = [(torch.empty(27, dtype=torch.float64, device="cuda"), torch.empty(27, dtype=torch.float64, device="cuda"))
            for _ in range(8)]
    for oa, ob in outs:
        with torch.cuda.stream(sa):
            hbl.moments_async(za, oa, n=n, stream=hbl.C.c_void_p(sa.cuda_stream))
        with torch.cuda.stream(sb):
            hbl.moments_async(zb, ob, n=n, stream=hbl.C.c_void_p(sb.cuda_stream))
    torch.cuda.synchronize()
    for oa, ob in outs:
        assert oa.cpu().tolist() == want_a[0] + want_a[1]
        assert ob.cpu().tolist() == want_b[0] + want_b[1]
    got = {}

    def sync_moments(key, z, st):
        torch.cuda.set_device(0)
        with torch.cuda.stream(st):
            got[key] = [hbl.moments(z, n=n, stream=hbl.C.c_void_p(st.cuda_stream)) for _ in range(4)]

    th = [threading.Thread(target=sync_moments, args=("a", za, sa)),
          threading.Thread(target=sync_moments, args=("b", zb, sb))]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert all(r == want_a for r in got["a"]) and all(r == want_b for r in got["b"])


def test_compare_full_size_constant_shift(hbl):
    """Properties that hold at any size, checked at 2.5e7 particles (the
    benchmark bunch; 95 particles per thread, so the four-at-a-time loop,
    the pair loop and the single tail all run): a test bunch equal to the
    reference shifted by a constant c_j per row has rms_j = |c_j|/sigma_j and
    centroid_j = c_j/sigma_j (sigma of the reference), and unchanged
    emittances."""
    torch = __import__("torch")
    n = 25_000_000
    sig = W.BunchSpec(1, 1).sigma
    zf = hbl.new_bunch(n)
    hbl.fill_gaussian(zf, 21, (0.0,) * 6, sig, n=n)
    shift = [0.25 * s for s in sig]
    shift[1] = -shift[1]
    zs = zf.clone()
    zs[:, :n] += torch.tensor(shift, dtype=torch.float64, device="cuda")[:, None]
    _, cov = hbl.moments(zf, n=n)
    sd = [math.sqrt(cov[j * 6 - j * (j - 1) // 2]) for j in range(6)]   # diagonal of the upper triangle
    r, c, e = hbl.compare(zs, zf, n=n)
    for j in range(6):
        # the shifted rows are rounded once (ulp of |z| ~ 4 sigma), so the
        # differences are c_j to ~1e-15 relative of sigma
        assert abs(r[j] - abs(shift[j]) / sd[j]) < 1e-12, (j, r[j])
        assert abs(c[j] - shift[j] / sd[j]) < 1e-12, (j, c[j])
    assert max(abs(x) for x in e) < 1e-12, e
