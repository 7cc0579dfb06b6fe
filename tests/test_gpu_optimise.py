"""The sequential plasma-lens optimisation (§4.4) on the GPU: with the
fine-step stages as the model, and on the surrogate chain (the paper's use)
checked against the fine-step stages.  From a mis-set start it must find
lenses that image each stage exit onto the next entrance (R12 -> 0, a
property of the optics that the emittance objective does not state) and
lower the final emittance."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def test_sequential_lens_optimisation_finds_imaging(orc):
    from paper_2402_17248_amd import hbl
    from paper_2402_17248_amd.optimize import chain_emittances, optimise_lenses
    n, nsub = 20_000, 300
    wl_of = lambda lenses: W.c5_lens_chain(lenses, n=n, nsub=nsub)
    wl = wl_of([W.LENS_START] * 3)
    z0 = hbl.new_bunch(n)
    hbl.fill_gaussian(z0, wl.bunch.seed, (0.0,) * 6, wl.bunch.sigma, n=n)
    stages = [hbl.element(s) for s in wl.beamline if not isinstance(s, list)]

    def apply(k, z, ref, pre, m):
        hbl.apply_stage(z, stages[k], ref, n=m, pre=pre)

    lenses, eps, report = optimise_lenses(wl_of, W.LENS_START, z0, n, apply,
                                          bounds=((0.5, 7.3), (0.5, 20.0)), max_evals=150)
    start = chain_emittances(wl_of([W.LENS_START] * 3), z0, n, apply)
    best = chain_emittances(wl_of(lenses), z0, n, apply)
    assert abs(best[-1] / eps[-1] - 1) < 1e-12           # the recorded path is the chain's
    assert best[-1] < 0.05 * start[-1]
    for p, f in lenses:
        M = np.ascontiguousarray(np.eye(6))
        orc.push(M, W.interstage_lens(p, f), orc.Ref.from_energy(11_000.0))
        assert abs(M[0, 3]) < 0.02                         # start: R12 = -0.53 m
    assert all(r["evaluations"] <= 150 + 4 for r in report)    # scipy may finish its last step


def test_moment_driven_lenses_preserve_emittance(orc):
    """Lenses set from the beam moments measured after each stage (centred,
    waist at the next entrance): the next stage sees a beam at a waist, and
    the emittance after stage 1 is kept through the chain (fine-step stages)."""
    from paper_2402_17248_amd import hbl
    from paper_2402_17248_amd.optimize import chain_emittances, chain_with_moment_lenses, twiss_from_moments
    n, nsub = 20_000, 300
    wl_of = lambda lenses: W.c5_lens_chain(lenses, n=n, nsub=nsub)
    wl = wl_of([W.LENS_START] * 3)
    z0 = hbl.new_bunch(n)
    hbl.fill_gaussian(z0, wl.bunch.seed, (0.0,) * 6, wl.bunch.sigma, n=n)
    stages = [hbl.element(s) for s in wl.beamline if not isinstance(s, list)]

    def apply(k, z, ref, pre, m):
        hbl.apply_stage(z, stages[k], ref, n=m, pre=pre)

    lenses, eps = chain_with_moment_lenses(wl_of, z0, n, apply, W.LENS_GAP_LENGTH / 2)
    assert chain_emittances(wl_of(lenses), z0, n, apply)[-1] == eps[-1]
    assert max(eps) < 1.2 * eps[0]
    # the beam entering each later stage is at a waist: |alpha| small
    ref = hbl.Ref.from_energy(wl.E_MeV)
    z = z0.clone()
    for k in range(3):
        apply(k, z, ref, hbl.Lattice(wl_of(lenses).beamline[2 * k], ref), n)
        w = z.clone()
        r = ref.copy()
        hbl.Lattice(wl_of(lenses).beamline[2 + 2 * k], r).push(w, r, n=n)
        _, cov = hbl.moments(w, n=n)
        _, alpha, _ = twiss_from_moments(cov)
        assert abs(alpha) < 1e-3, (k, alpha)


def test_lens_optimisation_on_surrogate_chain():
    """§4.4 as the paper uses it: the lenses are optimised on the surrogate
    chain (every stage a network trained here on fine-step pairs, briefly:
    2^18 pairs, 200 epochs, two trust-region rounds per interstage).  The
    lenses found are checked with the fine-step stages: the final emittance
    is more than 20x below the start's and within 15 % of the one the same
    optimisation reaches on the fine-step chain itself (measured: 8 %), and
    the surrogate chain's emittance after each stage is within 35 % of the
    fine-step chain's at those lenses (measured: 19-25 %; 10 % with the
    benchmark's training; before the trust-region rounds the networks,
    trained on widely mis-set lenses, were off by up to 5x there).  Imaging
    is not required here: the search box bounds the lens position, and the
    stage-by-stage optimum may sit on its edge with a slightly smaller
    emittance after the next stage than the imaging lens gives."""
    from paper_2402_17248_amd import hbl
    from paper_2402_17248_amd.optimize import chain_emittances, optimise_lenses, optimise_lenses_on_surrogates
    n = 1 << 15
    box = ((2.0, 7.0), (1.6, 4.0))
    wl_of = lambda lenses, m=n: W.c5_lens_chain(lenses, n=m)
    wl = wl_of([W.LENS_START] * 3)
    z0 = hbl.new_bunch(n)
    hbl.fill_gaussian(z0, wl.bunch.seed, (0.0,) * 6, wl.bunch.sigma, n=n)
    stages = [hbl.element(s) for s in wl.beamline if not isinstance(s, list)]

    def apply_fine(k, z, ref, pre, m):
        hbl.apply_stage(z, stages[k], ref, n=m, pre=pre)

    lenses, _, report, surs, _, _ = optimise_lenses_on_surrogates(
        wl_of, W.LENS_START, z0, n, box, 1 << 18, 200, lambda k: 400 + k, lambda k: 500 + k,
        lambda k: 600 + k, refine_rounds=2)

    def apply_sur(k, z, ref, pre, m):
        surs[k].apply(z, ref, n=m, pre=pre)

    fine_lenses, _, _ = optimise_lenses(wl_of, W.LENS_START, z0, n, apply_fine, bounds=box, max_evals=200)
    fine_at_sur = chain_emittances(wl_of(lenses), z0, n, apply_fine)
    fine_at_fine = chain_emittances(wl_of(fine_lenses), z0, n, apply_fine)
    sur_at_sur = chain_emittances(wl_of(lenses), z0, n, apply_sur)
    print(f"surrogate-chain lenses {lenses}, fine-step-chain lenses {fine_lenses}; eps_x after stages 1-4: "
          f"fine-step at surrogate lenses {fine_at_sur}, fine-step optimum {fine_at_fine}, surrogate chain "
          f"{sur_at_sur}", flush=True)
    start = chain_emittances(wl_of([W.LENS_START] * 3), z0, n, apply_fine)
    assert fine_at_sur[-1] < 0.05 * start[-1]
    assert fine_at_sur[-1] <= 1.15 * fine_at_fine[-1]
    for a, b in zip(sur_at_sur, fine_at_sur):
        assert abs(a / b - 1) < 0.35, (sur_at_sur, fine_at_sur)
