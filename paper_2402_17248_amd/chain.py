"""Staged beamline driver: a sequence of lattice segments and plasma stages
(§4, Fig. 1) pushed through libhbl on one stream with no host
synchronisation between segments.  Each stage is taken by the fine-step map
or, when a surrogate is attached, by the surrogate (§2: the hybrid
conventional + surrogate beamline)."""
from __future__ import annotations

from typing import List, Optional, Sequence

from . import hbl


def train_concurrently(jobs: Sequence, max_workers: int = 4):
    """Train several networks at once.  jobs: (network, inputs, outputs,
    n_pairs, keyword arguments of its train()).  Each training runs on a
    stream of its own, driven by a host thread of its own (the library call
    is synchronous and releases the interpreter): one batch-4096 step keeps
    only 64 workgroups busy, so independent trainings overlap on the GPU,
    and each one's host-side epoch shuffles run on their own core.  Every
    training is deterministic and touches only its own buffers, so the
    results equal those of sequential training bitwise.  The pairs must
    have been written on the current stream; the streams wait for it.
    Returns the loss curves in job order."""
    import ctypes
    from concurrent.futures import ThreadPoolExecutor

    import torch
    if not jobs:
        return []
    if len({id(j[0]) for j in jobs}) != len(jobs):
        raise ValueError("train_concurrently: a network appears in more than one job")
    main = torch.cuda.current_stream()
    device = torch.cuda.current_device()
    streams = [torch.cuda.Stream() for _ in jobs]
    for st in streams:
        st.wait_stream(main)

    def run(j):
        net, zin, zout, n_pairs, kw = jobs[j]
        torch.cuda.set_device(device)
        with torch.cuda.stream(streams[j]):
            return net.train(zin, zout, n_pairs, stream=ctypes.c_void_p(streams[j].cuda_stream), **kw)

    with ThreadPoolExecutor(max_workers=max(1, min(max_workers, len(jobs)))) as ex:
        curves = list(ex.map(run, range(len(jobs))))
    for st in streams:
        main.wait_stream(st)
    return curves


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

    def entry_ref(self, k: int) -> hbl.Ref:
        """Reference particle at the entrance of stage k (0-based)."""
        ref = hbl.Ref.from_energy(self.E_MeV)
        j = 0
        for kind, v in self.segments:
            if kind == "lattice":
                ref.s += v.length
                continue
            if j == k:
                return ref
            ref.gamma += v.dE_MeV / ref.mass_MeV
            ref.s += v.L
            j += 1
        raise IndexError(k)

    def stage(self, k: int) -> hbl.Element:
        return [v for kind, v in self.segments if kind == "stage"][k]

    def make_pairs(self, k: int, n_pairs: int, seed: int, sigma, stream=None):
        """Training pairs for stage k (§3, §4.1): a fresh Gaussian bunch tracked
        with fine-step stages to the entrance of stage k, then stage k with its
        input recorded.  Returns (inputs, outputs) device bunches."""
        zin = hbl.new_bunch(n_pairs)
        zout = hbl.new_bunch(n_pairs)
        hbl.fill_gaussian(zout, seed, (0.0,) * 6, sigma, n=n_pairs, stream=stream)
        self.run(zout, n=n_pairs, stop_before_stage=k, record=zin, stream=stream)
        return zin, zout

    def train_surrogates(self, n_pairs: int, sigma, pair_seed, init_seed, shuffle_seed, epochs: int,
                         batch=4096, lr=1e-3, lr_final=1e-5, train_frac=0.7, stages=None, log=None,
                         keep_best=False, concurrent=True):
        """Train one surrogate per stage, each on its own pairs (the paper
        trains one network per stage, §4.2).  Seeds are callables of the
        1-based stage number.  keep_best: as in Surrogate.train.
        concurrent: the stages' trainings run at the same time on streams
        of their own (train_concurrently; bitwise the same networks),
        otherwise one after another."""
        ks = list(range(self.stage_count) if stages is None else stages)
        kw = lambda k: dict(batch=batch, epochs=epochs, lr=lr, lr_final=lr_final, train_frac=train_frac,
                            shuffle_seed=shuffle_seed(k + 1), keep_best=keep_best)
        surs = {k: hbl.Surrogate(init_seed(k + 1)) for k in ks}
        if concurrent:
            pairs = {k: self.make_pairs(k, n_pairs, pair_seed(k + 1), sigma) for k in ks}
            curves = train_concurrently([(surs[k], *pairs[k], n_pairs, kw(k)) for k in ks])
            del pairs
        else:
            curves = []
            for k in ks:
                zin, zout = self.make_pairs(k, n_pairs, pair_seed(k + 1), sigma)
                curves.append(surs[k].train(zin, zout, n_pairs, **kw(k)))
                del zin, zout
        for k, curve in zip(ks, curves):
            surs[k].set_stage(self.stage(k), self.entry_ref(k))
            self.surrogates[k] = surs[k]
            if log:
                log(f"stage {k + 1}: trained {epochs} epochs, final (train, test) loss {curve[-1].tolist()}")
        return curves

    def passes(self):
        """Group the segments into bunch passes: each stage absorbs the lattice
        segment right before it (its entrance gap) and, for the last segment,
        the one right after it (the exit gap).  Items: ("lattice", L) or
        ("stage", (pre, k, stage, post))."""
        out, segs, i, k = [], self.segments, 0, 0
        while i < len(segs):
            kind, v = segs[i]
            if kind == "lattice" and not (i + 1 < len(segs) and segs[i + 1][0] == "stage"):
                out.append(("lattice", v))
                i += 1
                continue
            pre = None
            if kind == "lattice":
                pre, i = v, i + 1
            st = segs[i][1]
            i += 1
            post = None
            if i == len(segs) - 1 and segs[i][0] == "lattice":
                post, i = segs[i][1], i + 1
            out.append(("stage", (pre, k, st, post)))
            k += 1
        return out

    def run(self, z, n=None, use_surrogates=False, stop_before_stage: Optional[int] = None,
            record=None, fused=True, gaps_fused=True, stream=None) -> hbl.Ref:
        """Push z in place.  stop_before_stage=k stops at the entrance of stage k
        (0-based); with record given, stage k is then applied with the input
        recorded (training pairs).  gaps_fused runs each gap in its stage's
        kernel (one bunch pass per stage); fused=False pushes lattices element
        by element (comparator).  All variants give bitwise equal results."""
        ref = hbl.Ref.from_energy(self.E_MeV)
        for kind, v in self.passes():
            if kind == "lattice":
                v.push(z, ref, fused=fused, n=n, stream=stream)
                continue
            pre, k, st, post = v
            if not (gaps_fused and fused):
                if pre is not None:
                    pre.push(z, ref, fused=fused, n=n, stream=stream)
                pre = None
            stopping = stop_before_stage is not None and k == stop_before_stage
            if stopping:
                if record is not None:
                    hbl.apply_stage(z, st, ref, record=record, n=n, stream=stream, pre=pre)
                elif pre is not None:
                    pre.push(z, ref, n=n, stream=stream)
                return ref
            post_now = post if (gaps_fused and fused) else None
            if use_surrogates:
                sur = self.surrogates[k]
                if sur is None:
                    raise RuntimeError(f"stage {k} has no surrogate attached")
                sur.apply(z, ref, n=n, stream=stream, pre=pre, post=post_now)
            else:
                hbl.apply_stage(z, st, ref, n=n, stream=stream, pre=pre, post=post_now)
            if post is not None and post_now is None:
                post.push(z, ref, fused=fused, n=n, stream=stream)
        return ref
