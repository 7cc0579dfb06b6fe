"""Benchmark: particles/s through the staged beamline (4 plasma stages with
triplet + chicane gaps, 2.5e7 electrons) with every stage taken by its
neural-network surrogate, against the same beamline with the fine-step
stages, on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

A step is one pass of the hot path over one synthetic bunch with the bunch
resident in HBM: Gaussian fill, the staged chain (lattice gaps fused, stages
by surrogate inference), and the final moment reduction, all enqueued on
one stream.  Before timing, the four surrogates are trained on the GPU by
the library's own kernels (one per stage, 2^20 pairs each).  Prints one
JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3
BF16_PEAK_TFLOPS = 2500.0
MLP_FLOP_PER_PARTICLE = 2 * (6 * 64 + 64 * 64 + 64 * 64 + 64 * 6)   # 17,920: dense layers, FMA = 2


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=25_000_000)
    ap.add_argument("--epochs", type=int, default=300, help="training epochs per surrogate")
    ap.add_argument("--pairs", type=int, default=1 << 20)
    ap.add_argument("--fine-steps", type=int, default=2, help="timed steps of the fine-step path")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline leg")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--pmc-probe", action="store_true",
                    help="short run for hardware-counter passes: one plain device copy of 2 x 1 GiB "
                         "(calibration) and 3 launches of the surrogate inference kernel on the "
                         "benchmark bunch (untrained weights), then exit")
    return ap.parse_args()


def pmc_probe(args):
    """Short, deterministic launch sequence for rocprofv3 --pmc passes."""
    import torch

    import workloads as W
    from paper_2402_17248_amd import hbl

    torch.cuda.set_device(0)
    a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")      # 1 GiB
    b = torch.empty_like(a)
    b.copy_(a)                                                           # reads 1 GiB, writes 1 GiB
    torch.cuda.synchronize()
    wl = W.c5_chain(n=args.n)
    sur = hbl.Surrogate(W.mlp_init_seed(1))
    sig = wl.bunch.sigma
    sur.set_norm([0.0] * 6 + list(sig) + [0.0] * 6 + list(sig))
    z = hbl.new_bunch(wl.bunch.n)
    hbl.fill_gaussian(z, wl.bunch.seed, (0.0,) * 6, sig, n=wl.bunch.n)
    for _ in range(3):
        sur.apply(z, n=wl.bunch.n)
    torch.cuda.synchronize()
    log(f"pmc probe done: copy 1 GiB, 3 x k_mlp_infer on {wl.bunch.n} particles")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def time_events(torch, fn, iters):
    """Average duration of fn() by HIP events on torch's current stream, the
    stream every library call below is enqueued on."""
    s = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(iters):
        fn()
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / iters * 1e-3


def cpu_baseline(wl, chain, budget_s):
    """The oracle, as it stands, on a bounded sample of the same workload:
    the staged beamline with the trained surrogates evaluated by the oracle's
    FP64 network, serial, one core."""
    import numpy as np

    import oracle
    from paper_2402_17248_amd import hbl

    params = [s.get_params() for s in chain.surrogates]
    norms = [np.array(s.get_norm()) for s in chain.surrogates]
    sh = oracle.shape()

    def run(m):
        z = oracle.fill_gaussian(m, wl.bunch.seed, (0.0,) * 6, wl.bunch.sigma)
        ref = oracle.Ref.from_energy(wl.E_MeV)
        t0 = time.perf_counter()
        k = 0
        for seg in wl.beamline:
            if isinstance(seg, list):
                oracle.push(z, seg, ref)
            else:
                z = oracle.mlp_apply(sh, params[k], norms[k], z, mode=0)
                ref.gamma += seg.dE_MeV / ref.mass_MeV
                k += 1
        return time.perf_counter() - t0

    t_small = run(256) / 256
    m = int(max(256, min(wl.bunch.n, budget_s / max(t_small, 1e-12))))
    t = run(m)
    return {"value": m / t, "unit": "particles/s", "cores": 1, "kind": "oracle",
            "sample": f"first {m} particles of the {wl.bunch.n}-particle bunch through the full staged "
                      f"beamline (lattice gaps + 4 surrogate stages), serial FP64 oracle, {t:.1f} s"}


def main():
    args = parse()
    if args.pmc_probe:
        pmc_probe(args)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; there is no multi-GPU path "
                                   "(particles shard by index with no exchange but a 27-value "
                                   "moment merge; not built)", "n_gpus": args.gpus}), flush=True)
        sys.exit(2)
    import numpy as np
    import torch

    import workloads as W
    from paper_2402_17248_amd import hbl
    from paper_2402_17248_amd.chain import Chain

    torch.cuda.set_device(0)
    wl = W.c5_chain(n=args.n)
    n = wl.bunch.n
    chain = Chain(wl.beamline, wl.E_MeV)
    sig = wl.bunch.sigma
    log(f"workload {wl.name}: n={n}, {chain.stage_count} stages, {chain.n_elements()} element pushes/particle")

    # ---- train the four stage surrogates on the GPU (not timed as the metric)
    t0 = time.perf_counter()
    curves = chain.train_surrogates(args.pairs, sig, W.c5_pair_seed, W.mlp_init_seed, W.shuffle_seed,
                                    epochs=args.epochs, batch=W.TRAIN_BATCH, lr=W.TRAIN_LR, lr_final=1e-5,
                                    train_frac=W.TRAIN_FRAC, log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    n_train, _ = W.split_counts(args.pairs)
    train_samples = chain.stage_count * args.epochs * (n_train // W.TRAIN_BATCH) * W.TRAIN_BATCH
    log(f"training: {t_train:.1f} s for {chain.stage_count} surrogates "
        f"({train_samples / t_train:.3g} training samples/s incl. pair generation)")

    z = hbl.new_bunch(n)
    out27 = torch.empty(27, dtype=torch.float64, device="cuda")

    def step(use_sur):
        hbl.fill_gaussian(z, wl.bunch.seed, (0.0,) * 6, sig, n=n)
        chain.run(z, n=n, use_surrogates=use_sur)
        hbl.moments_async(z, out27, n=n)

    def timed(use_sur, steps, warmup):
        for _ in range(warmup):
            step(use_sur)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            step(use_sur)
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / steps

    dt_sur = timed(True, args.steps, args.warmup)
    log(f"surrogate chain: {dt_sur * 1e3:.3f} ms/step, {n / dt_sur:.4g} particles/s")
    dt_fine = timed(False, args.fine_steps, 1)
    log(f"fine-step chain: {dt_fine * 1e3:.3f} ms/step, {n / dt_fine:.4g} particles/s")

    # ---- accuracy of the surrogate chain against the fine-step chain, same input
    zs = hbl.new_bunch(n)
    hbl.fill_gaussian(zs, wl.bunch.seed, (0.0,) * 6, sig, n=n)
    chain.run(zs, n=n, use_surrogates=True)
    hbl.fill_gaussian(z, wl.bunch.seed, (0.0,) * 6, sig, n=n)
    chain.run(z, n=n, use_surrogates=False)
    rms, cen, eps_rel = hbl.compare(zs, z, n=n)
    log(f"surrogate vs fine-step chain: eps_rel x,y,t = {eps_rel}, rms/sigma = {rms}")
    del zs

    # ---- dominant kernel: surrogate inference, timed alone on the stream
    sur0 = chain.surrogates[0]
    hbl.fill_gaussian(z, wl.bunch.seed, (0.0,) * 6, sig, n=n)
    t_inf = time_events(torch, lambda: sur0.apply(z, n=n), max(3, args.steps))
    fine_stage = chain.stage(0)
    t_fs = time_events(torch, lambda: hbl.apply_stage(z, fine_stage, chain.entry_ref(0), n=n), 2)
    mfma_achieved = MLP_FLOP_PER_PARTICLE * n / t_inf / 1e12
    log(f"inference kernel: {t_inf * 1e3:.3f} ms per stage ({n / t_inf:.4g} particles/s); "
        f"fine-step stage kernel: {t_fs * 1e3:.3f} ms; single-stage speed-up {t_fs / t_inf:.1f}x")

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(wl, chain, args.cpu_seconds)
        log(f"cpu oracle: {cpu['value']:.4g} particles/s ({cpu['sample']})")

    line = {
        "metric": "particles/s through staged beamline: surrogate vs fine-step stage, same error",
        "value": n / dt_sur, "unit": "particles/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt_sur * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16+f64", "data": "synthetic",
        "config": {"workload": wl.name, "particles": n, "stages": chain.stage_count,
                   "stage_path": "surrogate (MLP 6-64-64-64-6 tanh)",
                   "element_pushes_per_particle": chain.n_elements(),
                   "training": {"pairs_per_stage": args.pairs, "epochs": args.epochs,
                                "batch": W.TRAIN_BATCH, "lr": W.TRAIN_LR, "lr_final": 1e-5,
                                "seconds_total": t_train,
                                "final_test_loss": [float(c[-1, 1]) for c in curves]}},
        "fine_step_path": {"value": n / dt_fine, "ms_per_step": dt_fine * 1e3, "nsub": fine_stage.nsub,
                           "speedup_surrogate": dt_fine / dt_sur},
        "accuracy_vs_fine_step": {"eps_rel_xyt": eps_rel, "rms_over_sigma": rms,
                                  "centroid_over_sigma": cen},
        "single_stage": {"inference_ms": t_inf * 1e3, "fine_step_ms": t_fs * 1e3,
                         "speedup": t_fs / t_inf},
        "particle_element_pushes_per_s": chain.n_elements() * n / dt_sur,
        "roofline": {"bound": "mfma", "achieved": mfma_achieved, "peak": BF16_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": mfma_achieved / BF16_PEAK_TFLOPS, "traffic": None,
                     "kernel": "k_mlp_infer (surrogate inference)"},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
