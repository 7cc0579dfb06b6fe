"""Staged beamline driver: a sequence of lattice segments and plasma stages
(§4, Fig. 1) pushed through libhbl on one stream with no host
synchronisation between segments.  Each stage is taken by the fine-step map
or, when a surrogate is attached, by the surrogate (§2: the hybrid
conventional + surrogate beamline)."""
from __future__ import annotations

from typing import List, Optional

from . import hbl


class Chain:
    def __init__(self, beamline, E_MeV: float):
        """beamline: list of segments, each a list of linear elements or one
        stage description (with L, n0_m3, dE_MeV, nsub)."""
        self.E_MeV = E_MeV
        self.segments = []        # ("lattice", Lattice) | ("stage", Element)
        ref = hbl.Ref.from_energy(E_MeV)
        for seg in beamline:
            if isinstance(seg, list):
                self.segments.append(("lattice", hbl.Lattice(seg, ref)))
            else:
                el = hbl.element(seg)
                self.segments.append(("stage", el))
                ref.gamma += el.dE_MeV / ref.mass_MeV
        self.stage_count = sum(1 for k, _ in self.segments if k == "stage")
        self.surrogates: List[Optional[object]] = [None] * self.stage_count

    def n_elements(self) -> int:
        """Particle-element pushes per particle (a stage counts as one)."""
        return sum(v.n_elem if k == "lattice" else 1 for k, v in self.segments)

    def run(self, z, n=None, use_surrogates=False, stop_before_stage: Optional[int] = None,
            record=None, fused=True, stream=None) -> hbl.Ref:
        """Push z in place.  stop_before_stage=k stops at the entrance of stage k
        (0-based); with record given, stage k is then applied with the input
        recorded (training pairs)."""
        ref = hbl.Ref.from_energy(self.E_MeV)
        k = 0
        for kind, v in self.segments:
            if kind == "lattice":
                v.push(z, ref, fused=fused, n=n, stream=stream)
                continue
            if stop_before_stage is not None and k == stop_before_stage:
                if record is not None:
                    hbl.apply_stage(z, v, ref, record=record, n=n, stream=stream)
                return ref
            if use_surrogates:
                sur = self.surrogates[k]
                if sur is None:
                    raise RuntimeError(f"stage {k} has no surrogate attached")
                sur.apply(z, ref, n=n, stream=stream)
            else:
                hbl.apply_stage(z, v, ref, n=n, stream=stream)
            k += 1
        return ref
