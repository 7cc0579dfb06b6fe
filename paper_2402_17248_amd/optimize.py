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
                    before_interstage: Optional[Callable[[int, list], None]] = None,
                    refine_rounds: int = 0, refine: Optional[Callable[[int, list, tuple], None]] = None,
                    shrink: float = 4.0):
    """Optimise the three interstage lenses one after another.

    wl_of_lenses(lenses) -> workload whose beamline is [T, S1, I1, S2, I2, S3, I3, S4, T];
    z0: device bunch (n particles) at the chain entrance, left untouched;
    apply_stage(k, z, ref, pre_lattice, n): push z through stage k (0-based)
    with the lattice `pre_lattice` fused before it (None for none), ref moved.
    before_interstage(k, lenses), if given, runs before lens k is optimised
    (lenses 0..k-1 final), e.g. to train the model of stage k + 1 around the
    current design.  Trust-region refinement: after the search over `bounds`,
    refine_rounds times the box shrinks by `shrink` around the lens found
    (clipped to `bounds`), refine(k, lenses, box) runs (e.g. to retrain the
    model of stage k + 1 on settings inside the box, where the optimum lies)
    and the search restarts from the lens found, inside the box.  Returns the
    lenses found, the horizontal emittance after each stage, and per
    interstage the evaluation count and wall time."""
    import numpy as np
    from scipy.optimize import minimize

    lenses = [tuple(start)] * 3
    wl = wl_of_lenses(lenses)
    ref = hbl.Ref.from_energy(wl.E_MeV)
    z = z0.clone()
    apply_stage(0, z, ref, hbl.Lattice(wl.beamline[0], ref), n)       # entrance triplet + stage 1
    eps = [emittance_x(z, n)]
    report = []
    (P_lo, P_hi), (F_lo, F_hi) = bounds
    for k in range(3):
        if before_interstage is not None:
            before_interstage(k, list(lenses))
        ref_k = ref.copy()
        evals = 0

        def search(box, x0, steps):
            (p_lo, p_hi), (f_lo, f_hi) = box

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

            x0 = np.array(x0)
            # the initial simplex steps inwards from edges of the box
            dp = steps[0] if x0[0] + steps[0] <= p_hi else -steps[0]
            df = steps[1] if x0[1] + steps[1] <= f_hi else -steps[1]
            res = minimize(objective, x0, method="Nelder-Mead",
                           options={"maxfev": max_evals, "xatol": xatol, "fatol": fatol_rel * objective(x0),
                                    "initial_simplex": np.array([x0, x0 + (dp, 0.0), x0 + (0.0, df)])})
            return (float(res.x[0]), float(res.x[1]))

        t0 = time.perf_counter()
        found = search(bounds, lenses[k], (0.5, 0.2))
        boxes = []
        for r in range(refine_rounds):
            hp = 0.5 * (P_hi - P_lo) / shrink ** (r + 1)
            hf = 0.5 * (F_hi - F_lo) / shrink ** (r + 1)
            box = ((max(P_lo, found[0] - hp), min(P_hi, found[0] + hp)),
                   (max(F_lo, found[1] - hf), min(F_hi, found[1] + hf)))
            boxes.append(box)
            lenses[k] = found
            if refine is not None:
                t1 = time.perf_counter()
                refine(k, list(lenses), box)
                t0 += time.perf_counter() - t1          # model building is not search time
            found = search(box, found, (0.5 * hp, 0.5 * hf))
        dt = time.perf_counter() - t0
        lenses[k] = found
        gap = wl_of_lenses(lenses).beamline[2 + 2 * k]
        apply_stage(k + 1, z, ref, hbl.Lattice(gap, ref), n)
        eps.append(emittance_x(z, n))
        report.append({"interstage": k + 1, "lens": lenses[k], "evaluations": evals, "seconds": dt,
                       "eps_x_after_next_stage": eps[-1], "refine_boxes": boxes})
        if log:
            log(f"interstage {k + 1}: lens at {lenses[k][0]:.4f} m, f = {lenses[k][1]:.4f} m after "
                f"{evals} evaluations ({dt:.2f} s); eps_x after stage {k + 2}: {eps[-1]:.4e} m")
    return lenses, eps, report


def optimise_lenses_on_surrogates(wl_of_lenses: Callable, start: Tuple[float, float], z0, n: int,
                                  bounds, n_pairs: int, epochs: int, pair_seed: Callable[[int], int],
                                  init_seed: Callable[[int], int], shuffle_seed: Callable[[int], int],
                                  n_settings: int = 8, refine_rounds: int = 2, seed: int = 7,
                                  max_evals: int = 200, log=None):
    """§4.4 on the fast surrogate chain: every stage is taken by a surrogate
    trained on fine-step pairs.  Before lens k is optimised, the surrogate of
    stage k + 1 is trained on pairs pooled over the lens's start and
    n_settings - 1 seeded settings in `bounds` (the earlier lenses at the
    values found: the inputs the optimiser will produce); after the search,
    each trust-region round retrains it on the lens found and n_settings - 1
    seeded settings inside the shrunken box around it and searches again
    there, so that the model is accurate where the optimum lies.  Seeds are
    callables of the 0-based stage.  Returns (lenses, emittances after each
    stage as the surrogate chain predicts them, per-interstage report,
    surrogates, training settings, training seconds)."""
    import numpy as np
    import torch

    rng = np.random.default_rng(seed)
    (p_lo, p_hi), (f_lo, f_hi) = bounds
    settings = [tuple(start)] + [(float(p), float(f)) for p, f in
                                 zip(rng.uniform(p_lo, p_hi, n_settings - 1), rng.uniform(f_lo, f_hi, n_settings - 1))]
    surs = [None] * 4
    t_train = [0.0]
    training_sets = [{"stage": 1, "settings": [tuple(start)]}]

    def train(k, lens_sets):
        t0 = time.perf_counter()
        surs[k] = train_stage_surrogate(wl_of_lenses, k, lens_sets, n_pairs, pair_seed(k), init_seed(k),
                                        shuffle_seed(k), epochs=epochs, log=log)
        torch.cuda.synchronize()
        t_train[0] += time.perf_counter() - t0

    def with_lens(k, lenses, s):
        return list(lenses[:k]) + [s] + [tuple(start)] * (2 - k)

    def before_interstage(k, lenses):
        training_sets.append({"stage": k + 2, "settings": list(settings)})
        train(k + 1, [with_lens(k, lenses, s) for s in settings])

    def refine(k, lenses, box):
        g = np.random.default_rng(seed + 100 * (k + 1) + len(training_sets))
        (a, b), (c, d) = box
        local = [lenses[k]] + [(float(p), float(f)) for p, f in
                               zip(g.uniform(a, b, n_settings - 1), g.uniform(c, d, n_settings - 1))]
        training_sets.append({"stage": k + 2, "box": box, "settings": local})
        train(k + 1, [with_lens(k, lenses, s) for s in local])

    def apply_sur(k, z, ref, pre, m):
        surs[k].apply(z, ref, n=m, pre=pre)

    train(0, [[tuple(start)] * 3])
    lenses, eps, report = optimise_lenses(wl_of_lenses, start, z0, n, apply_sur, bounds=bounds,
                                          max_evals=max_evals, log=log, before_interstage=before_interstage,
                                          refine_rounds=refine_rounds, refine=refine)
    return lenses, eps, report, surs, training_sets, t_train[0]


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
