"""Sequential optimisation of the plasma lenses between stages (§4.4): the
lens position and strength of interstage k are varied to minimise the
horizontal emittance after stage k + 1, then fixed, and so on down the
chain, each objective evaluated on the GPU through the library (one fused
interstage + stage pass and one moment reduction per evaluation).  The
stages are taken by surrogates (the paper's use) or by the fine-step map
(to check the result in full fidelity)."""
from __future__ import annotations

import math
import time
from typing import Callable, List, Optional, Sequence, Tuple

from . import hbl


def emittance_x(z, n) -> float:
    _, cov = hbl.moments(z, n=n)
    return hbl.emittances(cov)[0]


def optimise_lenses(wl_of_lenses: Callable[[Sequence[Tuple[float, float]]], object],
                    start: Tuple[float, float], z0, n: int,
                    apply_stage: Callable, bounds: Tuple[Tuple[float, float], Tuple[float, float]],
                    # bounds: ((position min, max), (focal length min, max))
                    max_evals: int = 200, xatol: float = 1e-3, fatol_rel: float = 1e-5, log=None,
                    before_interstage: Optional[Callable[[int, list], None]] = None):
    """Optimise the three interstage lenses one after another.

    wl_of_lenses(lenses) -> workload whose beamline is [T, S1, I1, S2, I2, S3, I3, S4, T];
    z0: device bunch (n particles) at the chain entrance, left untouched;
    apply_stage(k, z, ref, pre_lattice, n): push z through stage k (0-based)
    with the lattice `pre_lattice` fused before it (None for none), ref moved.
    before_interstage(k, lenses), if given, runs before lens k is optimised
    (lenses 0..k-1 final), e.g. to train the model of stage k + 1 around the
    current design.  Returns the lenses found, the horizontal emittance after
    each stage, the evaluation count and the wall time per interstage."""
    import numpy as np
    from scipy.optimize import minimize

    lenses = [tuple(start)] * 3
    wl = wl_of_lenses(lenses)
    ref = hbl.Ref.from_energy(wl.E_MeV)
    z = z0.clone()
    apply_stage(0, z, ref, hbl.Lattice(wl.beamline[0], ref), n)       # entrance triplet + stage 1
    eps = [emittance_x(z, n)]
    report = []
    for k in range(3):
        if before_interstage is not None:
            before_interstage(k, list(lenses))
        ref_k = ref.copy()
        (p_lo, p_hi), (f_lo, f_hi) = bounds
        evals = 0

        def objective(v):
            nonlocal evals
            p, f = float(v[0]), float(v[1])
            if not (p_lo <= p <= p_hi and f_lo <= f <= f_hi):
                return 1e30                     # outside the lens's travel / strength range
            evals += 1
            trial = list(lenses)
            trial[k] = (p, f)
            gap = wl_of_lenses(trial).beamline[2 + 2 * k]
            r = ref_k.copy()
            w = z.clone()
            apply_stage(k + 1, w, r, hbl.Lattice(gap, r), n)
            return emittance_x(w, n)

        t0 = time.perf_counter()
        res = minimize(objective, np.array(lenses[k]), method="Nelder-Mead",
                       options={"maxfev": max_evals, "xatol": xatol, "fatol": fatol_rel * objective(lenses[k]),
                                "initial_simplex": np.array([lenses[k], (lenses[k][0] + 0.5, lenses[k][1]),
                                                             (lenses[k][0], lenses[k][1] + 0.2)])})
        dt = time.perf_counter() - t0
        lenses[k] = (float(res.x[0]), float(res.x[1]))
        gap = wl_of_lenses(lenses).beamline[2 + 2 * k]
        apply_stage(k + 1, z, ref, hbl.Lattice(gap, ref), n)
        eps.append(emittance_x(z, n))
        report.append({"interstage": k + 1, "lens": lenses[k], "evaluations": evals, "seconds": dt,
                       "eps_x_after_next_stage": eps[-1]})
        if log:
            log(f"interstage {k + 1}: lens at {lenses[k][0]:.4f} m, f = {lenses[k][1]:.4f} m after "
                f"{evals} evaluations ({dt:.2f} s); eps_x after stage {k + 2}: {eps[-1]:.4e} m")
    return lenses, eps, report


def chain_emittances(wl, z0, n: int, apply_stage: Callable) -> List[float]:
    """Horizontal emittance after each stage of the chain `wl` (gaps fused
    into the following stage)."""
    ref = hbl.Ref.from_energy(wl.E_MeV)
    z = z0.clone()
    out = []
    for k in range(4):
        apply_stage(k, z, ref, hbl.Lattice(wl.beamline[2 * k], ref), n)
        out.append(emittance_x(z, n))
    return out


def train_stage_surrogate(wl_of_lenses: Callable, k: int, lens_sets: Sequence[Sequence[Tuple[float, float]]],
                          n_pairs: int, pair_seed: int, init_seed: int, shuffle_seed: int, epochs: int,
                          batch: int = 4096, lr: float = 1e-3, lr_final: float = 1e-5, log=None,
                          keep_best: int = 1):
    """A surrogate of stage k (0-based) trained on pairs pooled over several
    chain configurations (lens_sets: the three interstage lenses of each), so
    that the inputs an optimiser produces stay inside the training
    distribution (the paper's widened training set, §4.2).  n_pairs split
    evenly over the configurations; the fine-step map produces the pairs.
    keep_best as in hbl_train_cfg (default: the lowest test loss, since the
    test split mixes the configurations)."""
    import torch

    from .chain import Chain

    per = n_pairs // len(lens_sets)
    tot = per * len(lens_sets)
    zin = hbl.new_bunch(tot)
    zout = hbl.new_bunch(tot)
    for j, lenses in enumerate(lens_sets):
        wl = wl_of_lenses(list(lenses))
        chain = Chain(wl.beamline, wl.E_MeV)
        a, b = chain.make_pairs(k, per, pair_seed * 64 + j, wl.bunch.sigma)
        zin[:, j * per:(j + 1) * per] = a[:, :per]
        zout[:, j * per:(j + 1) * per] = b[:, :per]
        del a, b
    # interleave the configurations so that the 70/30 split sees all of them
    idx = torch.arange(tot, device=zin.device).view(len(lens_sets), per).t().reshape(-1)
    zin[:, :tot] = zin[:, idx]
    zout[:, :tot] = zout[:, idx]
    sur = hbl.Surrogate(init_seed)
    curve = sur.train(zin, zout, tot, batch=batch, epochs=epochs, lr=lr, lr_final=lr_final,
                      shuffle_seed=shuffle_seed, keep_best=keep_best)
    wl = wl_of_lenses(list(lens_sets[0]))
    chain = Chain(wl.beamline, wl.E_MeV)
    sur.set_stage(chain.stage(k), chain.entry_ref(k))
    if log:
        log(f"lens chain stage {k + 1}: surrogate trained on {tot} pairs over {len(lens_sets)} "
            f"configurations, final (train, test) loss {curve[-1].tolist()}")
    return sur


# --------------------------------------------------------------------------
# Moment-driven lens strength (§4: the lens, centred between the stages, takes
# its strength from the beam moments measured in the gap after each stage).
# The paper cites the rule without giving it; here it is derived for a thin
# lens of strength q = 1/f between two linear sections of the gap whose x-plane
# transfer matrices are M1 (stage exit -> lens) and M2 (lens -> next entrance).
# With S the x-plane covariance at the exit and L = M1 S M1^T at the lens, the
# lens gives L' = [[L11, L12 - q L11], [L12 - q L11, L22 - 2 q L12 + q^2 L11]]
# and the x-px correlation at the next entrance, row 0 of M2 times L' times
# row 1 of M2, is a quadratic in q; its zero puts the beam at a waist
# (alpha = 0) there.  Of the two roots the one with the smaller beam at the
# entrance is the refocusing one (the other leaves the beam almost
# collimated).  For pure drifts d1, d2 the root is the textbook
# f = beta_L / (a - alpha_L), a = (beta_L + sqrt(beta_L^2 - 4 d2^2)) / (2 d2),
# in the Twiss parameters at the lens.  The matrices come from pushing probe
# particles through the compiled gap (the chicane's dipoles focus weakly,
# which a drift model misses at the metre-scale beta functions in the gap).
def twiss_from_moments(cov21):
    """(beta, alpha, emittance) of the x plane from a 21-term covariance."""
    xx, xpx, pxpx = cov21[0], cov21[3], cov21[15]
    eps = math.sqrt(max(xx * pxpx - xpx * xpx, 0.0))
    return xx / eps, -xpx / eps, eps


def x_transfer(seq, ref) -> Tuple[Tuple[float, float], Tuple[float, float]]:
    """x-plane 2x2 transfer matrix of a linear element sequence at the
    reference `ref` (left unchanged), from three probe particles (origin,
    unit-scaled x, unit-scaled px) pushed through the library."""
    import torch

    h = 1e-3
    z = hbl.new_bunch(3)
    z.zero_()
    z[0, 1] = h
    z[3, 2] = h
    if len(seq):
        hbl.Lattice(seq, ref).push(z, ref.copy(), n=3)
    w = z[:, :3].cpu().double()
    col = lambda j: ((w[0, j] - w[0, 0]).item() / h, (w[3, j] - w[3, 0]).item() / h)
    (a, c), (b, d) = col(1), col(2)
    return (a, b), (c, d)


def waist_lens_strength(cov21, m1, m2) -> float:
    """Thin-lens strength q = 1/f that puts the x-plane beam of covariance
    cov21 (at the stage exit) at a waist after m1, the lens and m2."""
    s11, s12, s22 = cov21[0], cov21[3], cov21[15]
    (p, r), (u, v) = m1
    l11 = p * p * s11 + 2 * p * r * s12 + r * r * s22
    l12 = p * u * s11 + (p * v + r * u) * s12 + r * v * s22
    l22 = u * u * s11 + 2 * u * v * s12 + v * v * s22
    (a, b), (c, d) = m2
    qa = b * d * l11
    qb = -(a * d + b * c) * l11 - 2.0 * b * d * l12
    qc = a * c * l11 + (a * d + b * c) * l12 + b * d * l22
    if qa == 0.0:
        roots = [-qc / qb]
    else:
        disc = qb * qb - 4.0 * qa * qc
        if disc < 0.0:
            raise ValueError("no lens strength puts the beam at a waist at the next entrance")
        t = -0.5 * (qb + math.copysign(math.sqrt(disc), qb))
        roots = [t / qa] + ([qc / t] if t != 0.0 else [])

    def size(q):
        return a * a * l11 + 2 * a * b * (l12 - q * l11) + b * b * (l22 - 2 * q * l12 + q * q * l11)
    return min(roots, key=size)


def chain_with_moment_lenses(wl_of_lenses: Callable, z0, n: int, apply_stage: Callable, lens_pos: float):
    """Run the chain stage by stage; after each stage read back the moments,
    set the next lens (at lens_pos in the gap) by the waist rule, and
    continue.  Returns the lenses and the horizontal emittance after each
    stage."""
    start = [(lens_pos, 1.0)] * 3
    wl = wl_of_lenses(start)
    ref = hbl.Ref.from_energy(wl.E_MeV)
    z = z0.clone()
    apply_stage(0, z, ref, hbl.Lattice(wl.beamline[0], ref), n)
    lenses = list(start)
    eps = []
    for k in range(3):
        _, cov = hbl.moments(z, n=n)
        eps.append(hbl.emittances(cov)[0])
        gap = wl_of_lenses(lenses).beamline[2 + 2 * k]
        i = next(j for j, e in enumerate(gap) if e.kind == "thin_lens")
        q = waist_lens_strength(cov, x_transfer(gap[:i], ref), x_transfer(gap[i + 1:], ref))
        if abs(q) < 1e-12:
            raise ValueError("waist rule gives no lens (q = 0)")
        lenses[k] = (lens_pos, 1.0 / q)
        gap_lat = wl_of_lenses(lenses).beamline[2 + 2 * k]
        apply_stage(k + 1, z, ref, hbl.Lattice(gap_lat, ref), n)
    eps.append(emittance_x(z, n))
    return lenses, eps
