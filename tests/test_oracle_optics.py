"""Pins of the oracle's linear element maps (CPU only).

The oracle's closed-form maps are checked against what the mathematics fixes
independently of them: the matrix exponential of each element's linearised
equations of motion, symplecticity, reversibility, the thin-lens limit,
brute-force 6x6 products, and emittance / phase-space-volume invariance.
"""
import numpy as np
import pytest
from scipy.linalg import expm

import workloads as W

# coordinate order of the bunch rows
X, Y, T, PX, PY, PT = range(6)
GAMMA_1GEV = 1000.0 / 0.51099895


def oracle_matrix(orc, elems, gamma=GAMMA_1GEV):
    """Columns = images of the unit vectors (the maps are linear)."""
    z = np.ascontiguousarray(np.eye(6))
    orc.push(z, list(elems), orc.Ref(gamma=gamma))
    return z


def generator(e, gamma=GAMMA_1GEV):
    """Linearised vector field dz/ds = A z of one element (bunch-row order)."""
    bg = np.sqrt(gamma**2 - 1.0)
    beta = bg / gamma
    A = np.zeros((6, 6))
    A[X, PX] = 1.0
    A[Y, PY] = 1.0
    A[T, PT] = 1.0 / bg**2
    if e.kind == W.QUAD:
        A[PX, X] = -e.k
        A[PY, Y] = +e.k
    elif e.kind == W.SBEND:
        rho = e.L / e.angle
        A[PX, X] = -1.0 / rho**2
        A[PX, PT] = -1.0 / (rho * beta)
        A[T, X] = 1.0 / (rho * beta)
    return A


def symplectic_form():
    # canonical pairs (x,px), (y,py), (t,pt) in bunch-row order
    S = np.zeros((6, 6))
    for q, p in ((X, PX), (Y, PY), (T, PT)):
        S[q, p] = 1.0
        S[p, q] = -1.0
    return S


ELEMS = [W.drift(0.25), W.drift(1.0), W.quad(1.0, +1.0), W.quad(1.0, -1.0), W.quad(0.3, 2.0),
         W.quad(0.3, -2.0), W.sbend(0.5, 5e-3), W.sbend(0.5, -5e-3), W.sbend(2.0, 0.3),
         W.sbend(1.0, -1.1)]


@pytest.mark.parametrize("e", ELEMS, ids=lambda e: f"{e.kind}-L{e.L}-k{e.k}-a{e.angle}")
@pytest.mark.parametrize("gamma", [GAMMA_1GEV, 1.5, 40.0])
def test_element_equals_matrix_exponential(orc, e, gamma):
    M = oracle_matrix(orc, [e], gamma)
    R = expm(e.L * generator(e, gamma))
    assert np.allclose(M, R, rtol=0, atol=1e-13 * max(1.0, np.abs(R).max()))


@pytest.mark.parametrize("e", ELEMS + [W.lens(0.5), W.lens(-2.0)], ids=lambda e: e.kind)
def test_symplectic_and_unit_determinant(orc, e):
    M = oracle_matrix(orc, [e])
    S = symplectic_form()
    err = np.abs(M.T @ S @ M - S).max()
    assert err < 5e-15 * max(1.0, np.abs(M).max() ** 2)
    assert abs(np.linalg.det(M) - 1.0) < 1e-12


@pytest.mark.parametrize("e", [W.drift(0.7), W.quad(1.0, 1.0), W.quad(0.3, -2.0), W.sbend(0.5, 5e-3),
                               W.sbend(2.0, 0.3)], ids=lambda e: e.kind)
def test_reversibility(orc, e):
    """Running an element backwards (L -> -L, angle -> -angle) inverts it."""
    back = W.Element(e.kind, L=-e.L, k=e.k, angle=-e.angle)
    M = oracle_matrix(orc, [e])
    Mb = oracle_matrix(orc, [back])
    assert np.abs(Mb @ M - np.eye(6)).max() < 1e-14


def test_lens_inverse_and_thin_quad_limit(orc):
    f = 0.5
    M = oracle_matrix(orc, [W.lens(f)])
    Mi = oracle_matrix(orc, [W.lens(-f)])
    assert np.abs(Mi @ M - np.eye(6)).max() < 1e-15
    # a quad of length L and strength 1/(f L) tends to the lens as L -> 0,
    # with an O(L) remainder
    errs = []
    for L in (1e-2, 5e-3):
        Q = oracle_matrix(orc, [W.drift(-L / 2), W.quad(L, 1.0 / (f * L)), W.drift(-L / 2)])
        # the quad's focusing is +k in x and -k in y: a lens in x, anti-lens in y
        ref = M.copy()
        ref[PY, Y] = +1.0 / f
        errs.append(np.abs(Q - ref).max())
    assert errs[0] < 1e-2 and errs[1] < errs[0] / 1.8


def test_small_angle_bend_is_smooth(orc):
    """sbend -> drift as angle -> 0 (no 1/angle blow-up)."""
    D = oracle_matrix(orc, [W.drift(0.5)])
    for a in (1e-3, 1e-6, 1e-9):
        B = oracle_matrix(orc, [W.sbend(0.5, a)])
        R = expm(0.5 * generator(W.sbend(0.5, a)))
        assert np.abs(B - R).max() < 1e-14
        assert np.abs(B - D).max() < 2 * a


def test_brute_force_product_on_tiny_bunch(orc):
    """Element-by-element tracking through the 58-element lattice equals the
    explicit product of the 58 matrix exponentials applied to each particle."""
    lat = W.c2_lattice()
    z0 = orc.fill_gaussian(16, 77, sigma=W.BunchSpec(1, 1).sigma)
    z = z0.copy()
    orc.push(z, lat, orc.Ref(gamma=GAMMA_1GEV))
    P = np.eye(6)
    for e in lat:
        if e.kind == W.THIN_LENS:
            K = np.eye(6)
            K[PX, X] = K[PY, Y] = -1.0 / e.f
        else:
            K = expm(e.L * generator(e))
        P = K @ P
    sig = np.array(W.BunchSpec(1, 1).sigma)
    err = np.abs(z - P @ z0) / sig[:, None]
    assert err.max() < 1e-12


def test_emittance_conserved_through_fodo(orc):
    wl = W.c1_fodo()
    z = orc.fill_gaussian(wl.bunch.n, wl.bunch.seed, wl.bunch.mean, wl.bunch.sigma)
    _, c0 = orc.moments(z)
    e0 = orc.emittances(c0)
    orc.track(z, wl.beamline, orc.Ref.from_energy(wl.E_MeV))
    _, c1 = orc.moments(z)
    e1 = orc.emittances(c1)
    C1 = orc.cov_matrix(c1)
    for p, (q, m) in enumerate(((X, PX), (Y, PY), (T, PT))):
        kappa = C1[q, q] * C1[m, m] / e1[p] ** 2
        assert abs(e1[p] / e0[p] - 1.0) < 10 * kappa * 2.3e-16


def test_chicane_conserves_phase_space_volume_and_r56(orc):
    ch = W.chicane()
    M = oracle_matrix(orc, ch)
    assert abs(np.linalg.det(M) - 1.0) < 1e-13
    z = orc.fill_gaussian(4000, 5, sigma=W.BunchSpec(1, 1).sigma)
    _, c0 = orc.moments(z)
    orc.push(z, ch, orc.Ref(gamma=GAMMA_1GEV))
    _, c1 = orc.moments(z)
    d0 = np.linalg.det(orc.cov_matrix(c0))
    d1 = np.linalg.det(orc.cov_matrix(c1))
    assert abs(d1 / d0 - 1.0) < 1e-9
    # textbook small-angle chicane: R56 = L_tot/(beta gamma)^2 + 2 theta^2 (dL + 2/3 L_b)/beta^2
    bg = np.sqrt(GAMMA_1GEV**2 - 1)
    beta = bg / GAMMA_1GEV
    th, Lb, dL = 5e-3, 0.5, 1.0
    r56 = (4 * Lb + 3 * dL) / bg**2 + 2 * th**2 * (dL + 2.0 / 3.0 * Lb) / beta**2
    assert abs(M[T, PT] / r56 - 1.0) < 1e-3
    # sector-bend chicane: the residual dispersion R16, R26 is third order in
    # the bend angle (first-order terms cancel between the four dipoles)
    Mh = oracle_matrix(orc, W.chicane(angle=th / 2))
    for r in (X, PX):
        assert 7.5 < M[r, PT] / Mh[r, PT] < 8.5
