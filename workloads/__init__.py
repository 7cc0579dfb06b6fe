"""Seeded synthetic workloads for the hybrid beamline hot path.

This module only *describes* inputs: bunch shapes, seeds, beamline element
lists and stage parameters.  It holds none of the method's arithmetic (no
transfer maps, no physical constants, no random number generation); both the
HIP library binding and the CPU oracle read these plain descriptions and
turn them into their own data structures.

Sizes follow the paper's workloads (Sandberg et al. 2024, §4, Table 1 and
§4.3: GeV-class electron bunches of 1e4..1e7 particles), with the synthetic
Gaussian of the benchmark definition standing in for the paper's WarpX
bunches, which are not available.

Coordinates are (x, y, t, px, py, pt) relative to a reference particle, row
order 0..5 in every bunch array.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Tuple

# Element kinds (values shared by name only; each side maps them itself).
DRIFT = "drift"
QUAD = "quad"
SBEND = "sbend"
THIN_LENS = "thin_lens"
STAGE = "stage"

COORDS = ("x", "y", "t", "px", "py", "pt")


@dataclass(frozen=True)
class Element:
    kind: str
    L: float = 0.0        # length [m]
    k: float = 0.0        # quadrupole strength [m^-2], k > 0 focuses x
    angle: float = 0.0    # bend angle [rad]
    f: float = 0.0        # thin-lens focal length [m]
    chromatic: bool = False  # quad / thin lens: focusing scales with the particle's momentum


@dataclass(frozen=True)
class Stage:
    """Plasma accelerator stage (§4, Fig. 1): length, density, energy gain."""
    L: float              # [m]
    n0_m3: float          # plasma electron density [m^-3]
    dE_MeV: float         # reference energy gain over the stage [MeV]
    nsub: int             # fine-step substeps
    chirp: float = 0.0    # particle gain dE (1 + chirp t) with t its entry t [1/m]; 0 = uniform


@dataclass(frozen=True)
class BunchSpec:
    n: int
    seed: int
    mean: Tuple[float, ...] = (0.0,) * 6
    sigma: Tuple[float, ...] = (10e-6, 10e-6, 10e-6, 1e-4, 1e-4, 1e-3)


def drift(L):
    return Element(DRIFT, L=L)


def quad(L, k):
    return Element(QUAD, L=L, k=k)


def sbend(L, angle):
    return Element(SBEND, L=L, angle=angle)


def lens(f):
    return Element(THIN_LENS, f=f)


# Electron energies are TOTAL energies (1 GeV -> gamma ~ 1957).
E0_MeV = 1000.0


def fodo_cell() -> List[Element]:
    """One FODO cell: D 0.25, QF 1.0 (k=+1), D 0.5, QD 1.0 (k=-1), D 0.25."""
    return [drift(0.25), quad(1.0, +1.0), drift(0.5), quad(1.0, -1.0), drift(0.25)]


def chicane(L_bend=0.5, angle=5e-3, L_drift=1.0) -> List[Element]:
    """Four-dipole chicane (+a, -a, -a, +a) with drifts between the dipoles."""
    return [sbend(L_bend, +angle), drift(L_drift), sbend(L_bend, -angle), drift(L_drift),
            sbend(L_bend, -angle), drift(L_drift), sbend(L_bend, +angle)]


def triplet(chromatic: bool = False) -> List[Element]:
    """Matching quad triplet around a stage: Q(+2) D0.2 Q(-2) D0.2 Q(+2), quads 0.3 m."""
    q = lambda k: Element(QUAD, L=0.3, k=k, chromatic=chromatic)
    return [q(+2.0), drift(0.2), q(-2.0), drift(0.2), q(+2.0)]


# Interstage triplet strengths (m^-2): with the drifts of interstage(), the
# gap from one stage's exit to the next stage's entrance images point to point
# in both planes (R12 = R34 = 0 to ~1e-9 m) with magnification -1, so the beam
# leaving a stage enters the next one with the same size and divergence.
INTERSTAGE_K_OUTER = 2.366855065
INTERSTAGE_K_INNER = 4.411922003


def interstage() -> List[Element]:
    """Gap between two stages: D 6.0, triplet Q(+k_o) D0.2 Q(-k_i) D0.2 Q(+k_o)
    (quads 0.3 m), D 0.5, four-dipole chicane (5 m), D 0.5 -- 13.3 m, 15
    elements, mirror-symmetric about the triplet centre (chicane taken as a
    drift transversely)."""
    ko, ki = INTERSTAGE_K_OUTER, INTERSTAGE_K_INNER
    return ([drift(6.0), quad(0.3, +ko), drift(0.2), quad(0.3, -ki), drift(0.2), quad(0.3, +ko),
             drift(0.5)] + chicane() + [drift(0.5)])


# Plasma-lens interstage (§4.4: a plasma lens between stages whose position and
# strength are optimised): D(p), thin lens f, D(LENS_GAP_DRIFT - p), the
# four-dipole chicane (5 m), D 0.5 -- 13.3 m from one stage to the next, like
# interstage().  Taking the chicane as a drift, point-to-point imaging with
# magnification -1 puts the lens in the middle, p = 6.65 m, with f = 3.325 m.
LENS_GAP_DRIFT = 7.8
LENS_GAP_LENGTH = 13.3
LENS_START = (5.0, 3.0)        # (position m, focal length m): where the optimisation starts


def interstage_lens(p: float, f: float) -> List[Element]:
    return [drift(p), lens(f), drift(LENS_GAP_DRIFT - p)] + chicane() + [drift(0.5)]


def plasma_stage(dE_MeV=9000.0, nsub=2000) -> Stage:
    """0.3 m stage at n0 = 1e17 cm^-3 = 1e23 m^-3."""
    return Stage(L=0.3, n0_m3=1e23, dE_MeV=dE_MeV, nsub=nsub)


@dataclass
class Workload:
    name: str
    bunch: BunchSpec
    E_MeV: float
    # beamline: list of segments; a segment is either a list of Elements
    # (tracked by the lattice pusher) or a Stage.
    beamline: list = field(default_factory=list)
    note: str = ""


def c1_fodo(n=10_000, seed=1) -> Workload:
    return Workload("fodo_1e4", BunchSpec(n, seed), E0_MeV, [fodo_cell()],
                    "one FODO cell, 1 GeV, FP64 tracking")


def c2_lattice() -> List[Element]:
    return [e for _ in range(10) for e in fodo_cell()] + chicane() + [lens(0.5)]


def c2_fused(n=1_000_000, seed=2) -> Workload:
    return Workload("lattice58_1e6", BunchSpec(n, seed), E0_MeV, [c2_lattice()],
                    "10 FODO + chicane + thin lens (58 elements), fused vs unfused")


# Energy-correlated gain of the chromatic variant: 1 % more gain per 200 um
# of t (the bunch is 10 um long, so +-1.5e-3 of the gain over +-3 sigma).
C3_CHIRP_PER_M = 50.0


def c3_stage(n=1_000_000, seed=13, nsub=2000) -> Workload:
    return Workload("stage_1to10GeV_1e6", BunchSpec(n, seed), E0_MeV,
                    [triplet(), plasma_stage(9000.0, nsub), triplet()],
                    "triplet + fine-step stage 1->10 GeV + triplet")


def c3_chromatic(n=1_000_000, seed=13, nsub=2000, chirp=C3_CHIRP_PER_M) -> Workload:
    """C3 with energy-dependent optics: chromatic triplets and a stage whose
    gain varies linearly along the bunch (gain dE (1 + chirp t))."""
    st = Stage(L=0.3, n0_m3=1e23, dE_MeV=9000.0, nsub=nsub, chirp=chirp)
    return Workload("stage_chromatic_1to10GeV_1e6", BunchSpec(n, seed), E0_MeV,
                    [triplet(True), st, triplet(True)],
                    "chromatic triplet + chirped fine-step stage 1->10 GeV + chromatic triplet")


C3_PAIR_SEED = 3
C3_PAIR_N = 1 << 20
C4_INFER_SEED = 4
C4_INFER_N = 10_000_000


def c5_chain(n=25_000_000, seed=5, nsub=2000, n_stages=4) -> Workload:
    """[T] S1 [I] S2 [I] S3 [I] S4 [T]: T the matching triplet of the single
    stage, I the imaging interstage (triplet + chicane); stage k runs
    1+10(k-1) -> 11+10(k-1) GeV."""
    bl: list = [triplet()]
    for k in range(n_stages):
        bl.append(plasma_stage(10_000.0, nsub))
        bl.append(interstage() if k < n_stages - 1 else triplet())
    return Workload("chain4_2.5e7", BunchSpec(n, seed), E0_MeV, bl,
                    "4 plasma stages (+10 GeV each) joined by imaging triplet+chicane interstages")


def c5_lens_chain(lenses, n=25_000_000, seed=5, nsub=2000, widen=1.0) -> Workload:
    """The four-stage chain with plasma-lens interstages; lenses = three
    (position, focal length) pairs.  widen scales the transverse sigmas of the
    initial bunch (wider training inputs)."""
    bl: list = [triplet()]
    for k in range(4):
        bl.append(plasma_stage(10_000.0, nsub))
        bl.append(interstage_lens(*lenses[k]) if k < 3 else triplet())
    sig = BunchSpec(1, 1).sigma
    sig = tuple(v * (widen if j in (0, 1, 3, 4) else 1.0) for j, v in enumerate(sig))
    return Workload("chain4_lens", BunchSpec(n, seed, sigma=sig), E0_MeV, bl,
                    "4 plasma stages joined by plasma-lens + chicane interstages")


def c5_pair_seed(k: int) -> int:
    """Seed of the training-pair bunch for stage k (1-based) of the chain."""
    return 50 + k


def mlp_init_seed(k: int) -> int:
    return 100 + k


def shuffle_seed(k: int) -> int:
    return 200 + k


# Surrogate shape and training recipe (benchmark definition; §3 Eq. 3-4 and §4.2).
MLP_SHAPE = (6, 64, 3, 6)          # n_in, width, hidden layers, n_out
TRAIN_BATCH = 4096
TRAIN_LR = 1e-3
TRAIN_FRAC = 0.7
# Model selection on the 30 % test split: among the last quarter of the epochs
# whose test loss is within 10 % of the lowest, the parameters whose predicted
# test outputs have the x and y emittances closest to the true ones
# (hbl_train_cfg.keep_best = 2).
TRAIN_KEEP = 2
ADAM_BETAS = (0.9, 0.999)
ADAM_EPS = 1e-8


def split_counts(n_pairs: int, frac: float = TRAIN_FRAC) -> Tuple[int, int]:
    """70/30 train/test split (§3): the first round(frac*n) pairs train."""
    n_train = int(round(frac * n_pairs))
    return n_train, n_pairs - n_train
