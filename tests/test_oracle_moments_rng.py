"""Pins of the oracle's moments, emittances, paired metrics and Gaussian fill
(CPU only).  Moments are pinned to exact rational arithmetic; the fill to the
statistics of the normal distribution."""
import math
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

import workloads as W

X, Y, T, PX, PY, PT = range(6)


def exact_cov(z):
    n = z.shape[1]
    F = [[Fraction(float(v)) for v in row] for row in z]
    mean = [sum(r) / n for r in F]
    cov = np.empty((6, 6), dtype=object)
    for j in range(6):
        for k in range(6):
            cov[j, k] = sum((F[j][i] - mean[j]) * (F[k][i] - mean[k]) for i in range(n)) / n
    return mean, cov


@pytest.mark.parametrize("n,offset", [(7, 0.0), (33, 0.0), (33, 1e3)])
def test_moments_exact_vs_rationals(orc, n, offset):
    rng = np.random.default_rng(n)
    z = np.ascontiguousarray(rng.normal(size=(6, n)) * np.array([1e-5, 1e-5, 1e-5, 1e-4, 1e-4, 1e-3])[:, None]
                             + offset * np.array([1e-5, 0, 1e-5, 0, 1e-4, 0])[:, None])
    m, c21 = orc.moments(z)
    me, ce = exact_cov(z)
    C = orc.cov_matrix(c21)
    for j in range(6):
        assert abs(Fraction(m[j]) - me[j]) <= abs(me[j]) * Fraction(2 ** -52) + Fraction(1e-300)
        for k in range(6):
            scale = math.sqrt(float(ce[j, j]) * float(ce[k, k]))
            assert abs(float(Fraction(C[j, k]) - ce[j, k])) <= 4e-16 * scale


def test_emittance_vs_rational_determinant(orc):
    rng = np.random.default_rng(5)
    z = rng.normal(size=(6, 40))
    z[PX] = 0.999 * z[X] + 0.01 * z[PX]            # strongly correlated plane
    z = np.ascontiguousarray(z)
    _, c21 = orc.moments(z)
    e = orc.emittances(c21)
    _, ce = exact_cov(z)
    # emittance of the exactly-known covariance, rounded covariance entries
    C = orc.cov_matrix(c21)
    for p, (q, r) in enumerate(((X, PX), (Y, PY), (T, PT))):
        det = Fraction(C[q, q]) * Fraction(C[r, r]) - Fraction(C[q, r]) ** 2
        assert abs(e[p] - math.sqrt(det)) <= 2.3e-16 * e[p]
        true = math.sqrt(ce[q, q] * ce[r, r] - ce[q, r] ** 2)
        kappa = float(ce[q, q] * ce[r, r]) / true**2
        assert abs(e[p] / true - 1) <= 4 * kappa * 2.3e-16


def test_normalised_emittance_matches_paper_table(orc):
    """Table 1 (§4): sigma_x = 0.75 um, sigma_px = 1.33 m_e c -> eps_n = 1 mm mrad."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "paper_table1_staged_beam.txt")
    row = [l.split() for l in open(path) if l.strip() and not l.startswith("#")][0]
    sx, spx, eps_n = float(row[0]) * 1e-6, float(row[1]), float(row[2]) * 1e-6
    g = 1000.0 / 0.51099895
    bg = math.sqrt(g * g - 1)
    n = 200_000
    z = orc.fill_gaussian(n, 9, sigma=(sx, sx, 1e-7, spx / bg, spx / bg, 1e-4))
    _, c21 = orc.moments(z)
    en = orc.emittances(c21)[0] * bg
    assert abs(en / eps_n - 1) < 0.003 + 4 / math.sqrt(n)


def test_compare_metrics(orc):
    f = orc.fill_gaussian(1000, 3, sigma=W.BunchSpec(1, 1).sigma)
    rms, cen, er = orc.compare(f, f)
    assert np.all(rms == 0) and np.all(cen == 0) and np.all(er == 0)
    s = f.copy()
    s[X] += 2e-7                                      # rigid shift: centroid only
    rms, cen, er = orc.compare(s, f)
    _, c21 = orc.moments(f)
    sx = math.sqrt(c21[0])
    assert abs(rms[X] - 2e-7 / sx) < 1e-12 and abs(cen[X] - 2e-7 / sx) < 1e-12
    assert abs(er[0]) < 1e-12
    s = f.copy()
    s[PX] *= 1.01                                     # scaled momentum: emittance +1 %
    _, _, er = orc.compare(s, f)
    assert abs(er[0] - 0.01) < 1e-12


def test_fill_statistics(orc):
    n = 200_000
    mean = (1e-6, -2e-6, 0.0, 1e-5, 0.0, -1e-4)
    sig = W.BunchSpec(1, 1).sigma
    z = orc.fill_gaussian(n, 1234, mean, sig)
    u = (z - np.array(mean)[:, None]) / np.array(sig)[:, None]
    for j in range(6):
        assert abs(u[j].mean()) < 5 / math.sqrt(n)
        assert abs(u[j].var() - 1) < 5 * math.sqrt(2 / n)
        assert abs(stats.kurtosis(u[j])) < 5 * math.sqrt(24 / n)
        assert stats.kstest(u[j], "norm").pvalue > 1e-4
    c = np.corrcoef(u)
    assert np.abs(c - np.eye(6)).max() < 5 / math.sqrt(n)


def test_fill_index_addressing(orc):
    full = orc.fill_gaussian(1000, 7)
    part = orc.fill_gaussian(100, 7, i0=450)
    assert np.array_equal(part, full[:, 450:550])
    idx = np.array([999, 3, 3, 500])
    sel = orc.fill_gaussian(0, 7, idx=idx)
    assert np.array_equal(sel, full[:, idx])
    other = orc.fill_gaussian(1000, 8)
    assert np.abs(np.corrcoef(full[0], other[0])[0, 1]) < 0.15


def test_philox_words_uniform(orc):
    words = np.array([orc.philox([i, 0, 0, 0], [17, 0]) for i in range(4096)], dtype=np.uint64).ravel()
    counts = np.bincount((words >> np.uint64(24)).astype(np.int64), minlength=256)
    chi2 = ((counts - counts.mean()) ** 2 / counts.mean()).sum()
    assert stats.chi2.sf(chi2, 255) > 1e-4
    # a one-bit change of the counter changes about half of the output bits
    a = np.array(orc.philox([5, 0, 0, 0], [17, 0]), dtype=np.uint32)
    b = np.array(orc.philox([4, 0, 0, 0], [17, 0]), dtype=np.uint32)
    flips = sum(bin(int(v)).count("1") for v in (a ^ b))
    assert 40 < flips < 88


def test_epoch_permutation(orc):
    n = 5000
    p0 = orc.epoch_perm(n, 9, 0)
    p1 = orc.epoch_perm(n, 9, 1)
    assert np.array_equal(np.sort(p0), np.arange(n))
    assert not np.array_equal(p0, p1)
    # position of element 0 over many epochs is spread over the range
    firsts = np.array([orc.epoch_perm(64, 3, e)[0] for e in range(2000)])
    counts = np.bincount(firsts, minlength=64)
    chi2 = ((counts - counts.mean()) ** 2 / counts.mean()).sum()
    assert stats.chi2.sf(chi2, 63) > 1e-4
