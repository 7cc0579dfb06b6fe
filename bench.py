"""Benchmark: particles/s through the staged beamline (4 plasma stages with
triplet + chicane gaps, 2.5e7 electrons), surrogate stages vs fine-step
stages, on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

A step is one pass of the hot path over one synthetic bunch: Gaussian fill,
the staged chain, and the final moment reduction, all enqueued on one stream
with the bunch resident in HBM.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=25_000_000)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline leg")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def time_gpu(torch, fn, iters):
    """Average duration of fn() (launches on torch's current stream) by HIP events."""
    s = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(iters):
        fn()
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / iters * 1e-3


def cpu_baseline(W, wl, budget_s):
    """The oracle, as it stands, on a bounded sample of the same workload."""
    import numpy as np

    import oracle
    sig, seed = wl.bunch.sigma, wl.bunch.seed

    def run(m):
        z = oracle.fill_gaussian(m, seed, (0.0,) * 6, sig)
        t0 = time.perf_counter()
        oracle.track(z, wl.beamline, oracle.Ref.from_energy(wl.E_MeV))
        return time.perf_counter() - t0

    t_small = run(64) / 64
    m = int(max(64, min(wl.bunch.n, budget_s / max(t_small, 1e-9))))
    t = run(m)
    return {"value": m / t, "unit": "particles/s", "cores": 1, "kind": "oracle",
            "sample": f"first {m} particles of the {wl.bunch.n}-particle bunch through the full "
                      f"fine-step chain, serial FP64 oracle, {t:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only: there is no multi-GPU path "
                                   "(particles shard trivially; see the design notes)",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch

    import workloads as W
    from paper_2402_17248_amd import hbl
    from paper_2402_17248_amd.chain import Chain

    torch.cuda.set_device(0)
    wl = W.c5_chain(n=args.n)
    n = wl.bunch.n
    chain = Chain(wl.beamline, wl.E_MeV)
    z = hbl.new_bunch(n)
    out27 = torch.empty(27, dtype=torch.float64, device="cuda")
    sig = wl.bunch.sigma

    def step(use_sur=False):
        hbl.fill_gaussian(z, wl.bunch.seed, (0.0,) * 6, sig, n=n)
        chain.run(z, n=n, use_surrogates=use_sur)
        hbl.moments_async(z, out27, n=n)

    log(f"workload {wl.name}: n={n}, {chain.stage_count} stages, {chain.n_elements()} element pushes/particle")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    fine_pps = n / dt
    log(f"fine-step chain: {dt*1e3:.2f} ms/step, {fine_pps:.4g} particles/s")

    # dominant kernel: the fine-step stage on the bunch at stage-1 entrance
    stage_el = chain.segments[1][1]
    zs = z.clone()
    ref0 = hbl.Ref.from_energy(wl.E_MeV)
    t_stage = time_gpu(torch, lambda: hbl.apply_stage(zs, stage_el, ref0.copy(), n=n), max(2, args.steps))
    flops = 10.0 * stage_el.nsub * n
    achieved = flops / t_stage / 1e12
    log(f"stage kernel: {t_stage*1e3:.3f} ms, {achieved:.2f} TFLOP/s FP64 algorithmic")

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(W, wl, args.cpu_seconds)
        log(f"cpu oracle: {cpu['value']:.4g} particles/s ({cpu['sample']})")

    line = {
        "metric": "particles/s through staged beamline: surrogate vs fine-step stage, same error",
        "value": fine_pps, "unit": "particles/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": wl.name, "particles": n, "stages": chain.stage_count,
                   "stage_path": "fine-step", "nsub": stage_el.nsub,
                   "element_pushes_per_particle": chain.n_elements()},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS, "traffic": None,
                     "kernel": "k_stage (fine-step plasma stage)"},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
