"""Pins of the oracle's energy-dependent variants (CPU only): chromatic
quadrupoles and thin lenses (focusing strength k / (1 + delta), expanded to
first order in delta = -pt / beta), and the stage with an energy-correlated
gain (particle gain dE (1 + chirp t)).  The references are written
independently: the exact per-particle thick-quad map from the matrix
exponential of its own field, exact energy bookkeeping, and the
flight-time integral by quadrature."""
import math

import numpy as np
import pytest
from scipy import integrate
from scipy.linalg import expm

import workloads as W

MEC2 = 0.51099895
X, Y, T, PX, PY, PT = range(6)


def particles(pt_scale, n=12, seed=3):
    rng = np.random.default_rng(seed)
    z = np.zeros((6, n))
    z[X] = rng.normal(0, 1e-3, n)
    z[Y] = rng.normal(0, 1e-3, n)
    z[T] = rng.normal(0, 1e-5, n)
    z[PX] = rng.normal(0, 1e-3, n)
    z[PY] = rng.normal(0, 1e-3, n)
    z[PT] = rng.normal(0, pt_scale, n)
    return np.ascontiguousarray(z)


def beta_of(E):
    g = E / MEC2
    return math.sqrt(g * g - 1) / g


def exact_quad(z, L, k, beta):
    """Per particle, the plane maps of the field x'' = -k_i x, k_i = k / (1 + delta)."""
    out = z.copy()
    for i in range(z.shape[1]):
        d = -z[PT, i] / beta
        ki = k / (1 + d)
        Mx = expm(np.array([[0.0, 1.0], [-ki, 0.0]]) * L)
        My = expm(np.array([[0.0, 1.0], [ki, 0.0]]) * L)
        out[X, i], out[PX, i] = Mx @ np.array([z[X, i], z[PX, i]])
        out[Y, i], out[PY, i] = My @ np.array([z[Y, i], z[PY, i]])
    return out


@pytest.mark.parametrize("k", [2.0, -3.5])
def test_chromatic_quad_first_order_in_delta(orc, k):
    E, L = 1000.0, 0.3
    beta = beta_of(E)
    errs = []
    for s in (1e-3, 5e-4):
        z = particles(s)
        ref = exact_quad(z, L, k, beta)
        orc.push(z, [W.Element(W.QUAD, L=L, k=k, chromatic=True)], orc.Ref.from_energy(E))
        scale = np.abs(ref[[X, Y, PX, PY]]).max()
        errs.append(np.abs(z[[X, Y, PX, PY]] - ref[[X, Y, PX, PY]]).max() / scale)
        # the achromatic map misses a first-order term
        a = particles(s)
        orc.push(a, [W.Element(W.QUAD, L=L, k=k)], orc.Ref.from_energy(E))
        assert np.abs(a[[X, Y, PX, PY]] - ref[[X, Y, PX, PY]]).max() / scale > 20 * errs[-1]
    assert errs[0] < 5 * (1e-3 * 3) ** 2                   # second order in delta
    assert 3.0 < errs[0] / errs[1] < 5.0                   # halving delta quarters the error


def test_chromatic_lens_and_achromatic_limit(orc):
    E, f = 1000.0, 0.5
    beta = beta_of(E)
    z = particles(1e-3)
    z0 = z.copy()
    orc.push(z, [W.Element(W.THIN_LENS, f=f, chromatic=True)], orc.Ref.from_energy(E))
    d = -z0[PT] / beta
    exact = z0[PX] - z0[X] / (f * (1 + d))
    assert np.abs(z[PX] - exact).max() < 3 * np.abs(z0[X] / f * d * d).max() + 1e-18
    assert np.array_equal(z[X], z0[X])
    # zero energy deviation: the chromatic maps reduce to the achromatic ones
    for el in (W.Element(W.QUAD, L=0.3, k=2.0), W.Element(W.THIN_LENS, f=0.5)):
        a = particles(0.0)
        b = a.copy()
        orc.push(a, [el], orc.Ref.from_energy(E))
        orc.push(b, [W.Element(el.kind, L=el.L, k=el.k, f=el.f, chromatic=True)], orc.Ref.from_energy(E))
        assert np.array_equal(a, b)


def test_chirped_stage_energy_and_flight_time(orc):
    """pt out from energy bookkeeping: E_i,out = E_i,in + dE (1 + chirp t_i);
    t out from the first-order flight-time integral."""
    E, dE, L, chirp, nsub = 1000.0, 9000.0, 0.3, 80.0, 300
    z = particles(1e-3)
    z0 = z.copy()
    st = W.Stage(L=L, n0_m3=1e23, dE_MeV=dE, nsub=nsub, chirp=chirp)
    ref = orc.Ref.from_energy(E)
    orc.push(z, [st], ref)
    g_in, g_out = E / MEC2, (E + dE) / MEC2
    bg_in, bg_out = math.sqrt(g_in**2 - 1), math.sqrt(g_out**2 - 1)
    # energies in units of m c^2; pt = -(gamma_i - gamma_ref) / (beta gamma)_ref
    gi_in = g_in - z0[PT] * bg_in
    gi_out = gi_in + (dE / MEC2) * (1 + chirp * z0[T])
    # the bookkeeping subtracts energies of ~2e4 m c^2: its own rounding is ~1e-16 g_out / bg_out
    assert np.abs(z[PT] + (gi_out - g_out) / bg_out).max() < 16 * 2.2e-16 * g_out / bg_out
    assert np.abs(z[PT] - z0[PT] * bg_in / bg_out).max() > 1e-6          # the chirp matters
    gp = (g_out - g_in) / L
    for i in range(z.shape[1]):
        dgam = lambda s: (gi_in[i] - g_in) + gp * chirp * z0[T, i] * s    # gamma_i - gamma_ref
        dt = integrate.quad(lambda s: -dgam(s) / (g_in + gp * s) ** 3, 0, L, epsabs=0, epsrel=1e-12)[0]
        assert abs(z[T, i] - z0[T, i] - dt) < 1e-9 * abs(dt) + 1e-24


def test_chirped_stage_is_the_stage_of_the_particle_own_gain(orc):
    """Transversely, a particle at fixed t through the chirped stage moves as
    through an unchirped stage of gain dE (1 + chirp t): same x, y and the same
    u = px * (beta gamma)_ref,out once each side's exit reference is undone."""
    E, dE, L, chirp, nsub = 1000.0, 9000.0, 0.3, 80.0, 400
    z = particles(1e-3, n=6)
    for i in range(z.shape[1]):
        one = np.ascontiguousarray(z[:, i:i + 1])
        a = one.copy()
        orc.push(a, [W.Stage(L=L, n0_m3=1e23, dE_MeV=dE, nsub=nsub, chirp=chirp)], orc.Ref.from_energy(E))
        dEi = dE * (1 + chirp * one[T, 0])
        b = one.copy()
        orc.push(b, [W.Stage(L=L, n0_m3=1e23, dE_MeV=dEi, nsub=nsub)], orc.Ref.from_energy(E))
        bg_a = math.sqrt(((E + dE) / MEC2) ** 2 - 1)
        bg_b = math.sqrt(((E + dEi) / MEC2) ** 2 - 1)
        for j in (X, Y):
            assert abs(a[j, 0] - b[j, 0]) < 1e-12 * np.abs(one[[X, Y]]).max()
        for j in (PX, PY):
            assert abs(a[j, 0] * bg_a - b[j, 0] * bg_b) < 1e-12 * np.abs(one[[PX, PY]]).max() * bg_b * 30
