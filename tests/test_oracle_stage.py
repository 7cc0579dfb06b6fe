"""Pins of the oracle's fine-step plasma stage (CPU only).

Linear ion-channel focusing du/ds = -kappa x, dx/ds = u / gamma_i(s), with
gamma_i ramping linearly.  Pinned against closed forms that do not share the
integrator's steps: the Chebyshev power of a unimodular 2x2 matrix (no ramp),
the continuous cos/sin solution, the Bessel solution of the ramped equation,
the matched-beam scaling laws of the paper (§4), the determinant of the
transverse Jacobian, the flight-time integral, and time reversal.
"""
import math
import os

import numpy as np
import pytest
from scipy import integrate, special

import workloads as W

MEC2 = 0.51099895
QE, EPS0, ME, CL = 1.602176634e-19, 8.8541878128e-12, 9.1093837015e-31, 299792458.0
X, Y, T, PX, PY, PT = range(6)
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def kappa(n0):
    return 0.5 * n0 * QE**2 / (EPS0 * ME * CL**2)


def run_stage(orc, z, E_MeV, dE, nsub, L=0.3, n0=1e23):
    ref = orc.Ref.from_energy(E_MeV)
    orc.push(z, [W.Stage(L=L, n0_m3=n0, dE_MeV=dE, nsub=nsub)], ref)
    return ref


def probe_particles(n=8, seed=11):
    rng = np.random.default_rng(seed)
    z = np.zeros((6, n))
    z[X] = rng.normal(0, 10e-6, n)
    z[Y] = rng.normal(0, 10e-6, n)
    z[PX] = rng.normal(0, 1e-4, n)
    z[PY] = rng.normal(0, 1e-4, n)
    z[PT] = rng.normal(0, 1e-3, n)
    return np.ascontiguousarray(z)


def test_kp_value():
    # n0 = 1e17 cm^-3: k_p = omega_p / c = 5.95e4 m^-1
    assert abs(math.sqrt(2 * kappa(1e23)) / 5.9507e4 - 1) < 1e-4


def test_no_ramp_equals_chebyshev_power(orc):
    """Without energy gain the N-step map is the N-th power of one
    unimodular step matrix T:  T^N = cos(N phi) I + sin(N phi)/sin(phi) (T - cos(phi) I)."""
    E, N, L = 1000.0, 2000, 0.3
    z0 = probe_particles()
    z = z0.copy()
    run_stage(orc, z, E, 0.0, N, L)
    g0 = E / MEC2
    bg = math.sqrt(g0**2 - 1)
    h, kap = L / N, kappa(1e23)
    for i in range(z0.shape[1]):
        gi = g0 - z0[PT, i] * bg
        Tm = np.array([[1 - h * h * kap / (2 * gi), h / gi],
                       [-h * kap * (1 - h * h * kap / (4 * gi)), 1 - h * h * kap / (2 * gi)]])
        c = 0.5 * np.trace(Tm)
        phi = math.acos(c)
        P = math.cos(N * phi) * np.eye(2) + math.sin(N * phi) / math.sin(phi) * (Tm - c * np.eye(2))
        for (q, p) in ((X, PX), (Y, PY)):
            xin = np.array([z0[q, i], z0[p, i] * bg])
            xo = P @ xin
            # rounding accumulates over N steps: compare on the scale of the
            # oscillation amplitude of each variable
            wg = math.sqrt(kap * gi)
            amp_x = math.hypot(xin[0], xin[1] / wg)
            amp_u = math.hypot(xin[1], xin[0] * wg)
            assert abs(z[q, i] - xo[0]) < N * 1e-15 * amp_x
            assert abs(z[p, i] * bg - xo[1]) < N * 1e-15 * amp_u


def test_no_ramp_converges_to_harmonic_solution(orc):
    E, L = 1000.0, 0.3
    z0 = probe_particles()
    g0 = E / MEC2
    bg = math.sqrt(g0**2 - 1)
    kap = kappa(1e23)
    errs = []
    for N in (8000, 16000, 32000):
        z = z0.copy()
        run_stage(orc, z, E, 0.0, N, L)
        gi = g0 - z0[PT] * bg
        w = np.sqrt(kap / gi)
        u0 = z0[PX] * bg
        x_exact = z0[X] * np.cos(w * L) + u0 / (gi * w) * np.sin(w * L)
        errs.append(np.abs(z[X] - x_exact).max())
    assert 3.6 < errs[0] / errs[1] < 4.4 and 3.6 < errs[1] / errs[2] < 4.4


def bessel_solution(x0, u0, ga, gb, kap, gp):
    """x(gamma) = A J0(z) + B Y0(z), z = 2 sqrt(kap gamma)/gp, u = gp gamma dx/dgamma."""
    def basis(g):
        zz = 2.0 * np.sqrt(kap * g) / gp
        xr = np.array([special.j0(zz), special.y0(zz)])
        ur = -0.5 * gp * zz * np.array([special.j1(zz), special.y1(zz)])
        return xr, ur
    xa, ua = basis(ga)
    AB = np.linalg.solve(np.array([xa, ua]), np.array([x0, u0]))
    xb, ub = basis(gb)
    return xb @ AB, ub @ AB


def test_ramp_converges_to_bessel_solution(orc):
    E, dE, L = 1000.0, 9000.0, 0.3
    z0 = probe_particles()
    g_in = E / MEC2
    g_out = (E + dE) / MEC2
    bg_in, bg_out = math.sqrt(g_in**2 - 1), math.sqrt(g_out**2 - 1)
    kap, gp = kappa(1e23), (g_out - g_in) / L
    ref_x = np.empty(z0.shape[1])
    ref_u = np.empty(z0.shape[1])
    for i in range(z0.shape[1]):
        dg = -z0[PT, i] * bg_in
        ref_x[i], ref_u[i] = bessel_solution(z0[X, i], z0[PX, i] * bg_in, g_in + dg, g_out + dg, kap, gp)
    errs = []
    for N in (2000, 4000, 8000):
        z = z0.copy()
        ref = run_stage(orc, z, E, dE, N, L)
        assert abs(ref.gamma - g_out) < 1e-12 * g_out and abs(ref.s - L) < 1e-15
        errs.append(max(np.abs(z[X] - ref_x).max() / 1e-5, np.abs(z[PX] * bg_out - ref_u).max() / np.abs(ref_u).max()))
    assert errs[2] < 2e-3
    assert 3.8 < errs[0] / errs[1] < 4.2 and 3.8 < errs[1] / errs[2] < 4.2


def load_exponents():
    ex = {}
    with open(os.path.join(GOLDEN, "matched_beam_scaling.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                k, v = line.split()
                ex[k] = float(v)
    return ex


def test_matched_beam_scaling(orc):
    """Matched beam: sigma_x ~ E^(-1/4), divergence ~ E^(-3/4) (§4)."""
    ex = load_exponents()
    E, dE = 1000.0, 9000.0
    g_in, g_out = E / MEC2, (E + dE) / MEC2
    bg_in = math.sqrt(g_in**2 - 1)
    # matched (adiabatic) beam of the ramped channel: beta = 1/sqrt(K) =
    # sqrt(gamma/kappa); the envelope shrinks as gamma^(-1/4), so
    # <x x'> = sigma^2 d(ln sigma)/ds fixes alpha = beta g'/(4 gamma)
    kap = kappa(1e23)
    beta_m = math.sqrt(g_in / kap)
    alpha_m = ((g_out - g_in) / 0.3) / (4 * math.sqrt(g_in * kap))
    M = 64                                         # ring of equally spaced phases
    phi = 2 * np.pi * np.arange(M) / M
    a = 1e-6
    z = np.zeros((6, M))
    z[X] = a * np.cos(phi)
    z[PX] = -(a / beta_m) * (alpha_m * np.cos(phi) + np.sin(phi)) * g_in / bg_in
    z = np.ascontiguousarray(z)
    s_in = (np.sqrt(np.mean(z[X] ** 2)), np.sqrt(np.mean(z[PX] ** 2)))
    run_stage(orc, z, E, dE, 16000)
    s_out = (np.sqrt(np.mean(z[X] ** 2)), np.sqrt(np.mean(z[PX] ** 2)))
    r = g_out / g_in
    # WKB (adiabatic) error of the scaling laws is second order in g'/(gamma sqrt(K))
    assert abs(s_out[0] / s_in[0] / r ** ex["sigma_x"] - 1) < 1e-4
    assert abs(s_out[1] / s_in[1] / r ** ex["sigma_theta_x"] - 1) < 1e-4


def test_transverse_jacobian_determinant(orc):
    """At fixed energy offset the (x, px) map is linear with det = bg_in/bg_out
    (KDK is symplectic in (x, u); px = u / (beta gamma)_ref)."""
    E, dE = 1000.0, 9000.0
    for pt in (0.0, 2e-3, -3e-3):
        z = np.zeros((6, 3))
        z[PT] = pt
        z[X, 1] = 1e-5
        z[PX, 2] = 1e-4
        z = np.ascontiguousarray(z)
        run_stage(orc, z, E, dE, 2000)
        J = np.array([[(z[X, 1] - z[X, 0]) / 1e-5, (z[X, 2] - z[X, 0]) / 1e-4],
                      [(z[PX, 1] - z[PX, 0]) / 1e-5, (z[PX, 2] - z[PX, 0]) / 1e-4]])
        g_in, g_out = E / MEC2, (E + dE) / MEC2
        want = math.sqrt(g_in**2 - 1) / math.sqrt(g_out**2 - 1)
        assert abs(np.linalg.det(J) / want - 1) < 1e-9


def test_longitudinal_map(orc):
    """pt scales by bg_in/bg_out (same energy gain for all particles) and the
    flight-time term equals bg_in * integral ds / gamma_ref(s)^3."""
    E, dE, L = 1000.0, 9000.0, 0.3
    z = probe_particles()
    z0 = z.copy()
    run_stage(orc, z, E, dE, 100, L)
    g_in, g_out = E / MEC2, (E + dE) / MEC2
    bg_in, bg_out = math.sqrt(g_in**2 - 1), math.sqrt(g_out**2 - 1)
    assert np.allclose(z[PT], z0[PT] * bg_in / bg_out, rtol=1e-15, atol=0)
    r56 = bg_in * integrate.quad(lambda s: (g_in + (g_out - g_in) * s / L) ** -3, 0, L, epsabs=0, epsrel=1e-13)[0]
    assert np.allclose(z[T] - z0[T], r56 * z0[PT], rtol=1e-9, atol=1e-30)


def test_monoenergetic_emittance_conserved(orc):
    """All particles at the reference energy: the stage is linear and
    symplectic in (x, u), so the normalised emittance is conserved."""
    z = orc.fill_gaussian(4000, 21, sigma=(10e-6, 10e-6, 10e-6, 1e-4, 1e-4, 0.0))
    g_in = 1000.0 / MEC2
    _, c0 = orc.moments(z)
    e0 = orc.emittances(c0)[:2] * math.sqrt(g_in**2 - 1)
    ref = run_stage(orc, z, 1000.0, 9000.0, 2000)
    _, c1 = orc.moments(z)
    e1 = orc.emittances(c1)[:2] * math.sqrt(ref.gamma**2 - 1)
    C1 = orc.cov_matrix(c1)
    for p, (q, m) in enumerate(((X, PX), (Y, PY))):
        kap = C1[q, q] * C1[m, m] / (e1[p] / math.sqrt(ref.gamma**2 - 1)) ** 2
        assert abs(e1[p] / e0[p] - 1) < 2000 * 10 * kap * 2.3e-16 + 1e-12


def test_chromatic_stage_grows_emittance(orc):
    """With 1e-3 energy spread each particle rotates by its own phase: the
    mismatched beam filaments and its emittance grows."""
    wl = W.c3_stage(n=4000)
    z = orc.fill_gaussian(wl.bunch.n, wl.bunch.seed, wl.bunch.mean, wl.bunch.sigma)
    ref = orc.Ref.from_energy(wl.E_MeV)
    orc.push(z, wl.beamline[0], ref)
    _, c0 = orc.moments(z)
    en0 = orc.emittances(c0)[0] * math.sqrt(ref.gamma**2 - 1)
    orc.push(z, [wl.beamline[1]], ref)
    _, c1 = orc.moments(z)
    en1 = orc.emittances(c1)[0] * math.sqrt(ref.gamma**2 - 1)
    assert en1 > 10 * en0


@pytest.mark.parametrize("nsub", [200, 2000])
def test_time_reversal(orc, nsub):
    """The kick-drift-kick step with the ramp evaluated at each substep's
    midpoint is time-symmetric: reversing the transverse momenta and running
    the decelerating stage (gamma_out -> gamma_in over the same length and
    substeps) returns every particle to its start, for any step count.  A
    ramp sampled at the substep ends, or an asymmetric split of the kicks,
    breaks this.  pt returns exactly (both stages rescale by a ratio of
    beta*gamma); t picks up the two first-order flight-time terms."""
    E, dE = 1000.0, 9000.0
    z = probe_particles(n=16, seed=5)
    z[PT] *= 10.0                      # strongly chromatic: phase depends on pt
    z0 = z.copy()
    ref = run_stage(orc, z, E, dE, nsub)
    t_fwd = z[T] - z0[T]
    z[PX] *= -1
    z[PY] *= -1
    run_stage(orc, z, E + dE, -dE, nsub)
    z[PX] *= -1
    z[PY] *= -1
    # inside the channel the angles reach ~x/beta ~ 1e-2, a hundred times the entrance
    # spread, so px, py return to ~1e-14 of their internal scale
    for j, s in ((X, 10e-6), (Y, 10e-6), (PX, 1e-2), (PY, 1e-2)):
        assert np.abs(z[j] - z0[j]).max() < 1e-13 * s, j
    # one substep more on the way back (a different midpoint grid) does not return
    w = z0.copy()
    run_stage(orc, w, E, dE, nsub)
    w[PX] *= -1
    w[PY] *= -1
    run_stage(orc, w, E + dE, -dE, nsub + 1)
    assert np.abs(w[X] - z0[X]).max() > 1e3 * 1e-13 * 10e-6
    assert np.allclose(z[PT], z0[PT], rtol=4e-16, atol=0)
    # t: each pass adds R56 * pt_at_entry, and R56_back * pt_out = R56 * pt_in here
    assert np.allclose(z[T] - z0[T], 2 * t_fwd, rtol=1e-12, atol=1e-30)
