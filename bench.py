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
# fused lattice pass: reads the 6 FP64 coordinates, writes the 5 a lattice element can change
# (no element changes pt)
LATTICE_BYTES = 88.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3
BF16_PEAK_TFLOPS = 2500.0
MLP_FLOP_PER_PARTICLE = 2 * (6 * 64 + 64 * 64 + 64 * 64 + 64 * 6)   # 17,920: dense layers, FMA = 2
# VALU issue: 256 CUs x 4 SIMDs x 32 lanes x 2.4 GHz full-rate FP32 lane-slots; a
# transcendental (exp2, reciprocal) issues at quarter rate and costs 4 slots.
VALU_PEAK_TSLOTS = 256 * 4 * 32 * 2.4e9 / 1e12                      # 78.6 T slots/s
# tanh(a) = 1 - 2/(2^(c a) + 1): exp2 (4) + add (1) + reciprocal (4) + fma (1) = 10 slots,
# 3 hidden layers x 64 activations per particle
ALU_SLOTS_PER_PARTICLE = 3 * 64 * 10                                 # 1,920
# HBM bytes per launch of the dominant kernel from the FETCH_SIZE / WRITE_SIZE counter
# runs of `--pmc-probe` (FETCH scaled x2.0, WRITE x1.0 by a 1 GiB device copy), averaged
# over its eight launches on 2.5e7 particles; to be re-taken whenever the kernel changes.
TRAFFIC_BYTES_PER_LAUNCH = 2.4004e9


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=25_000_000)
    ap.add_argument("--epochs", type=int, default=1200, help="training epochs per surrogate")
    ap.add_argument("--pairs", type=int, default=1 << 20)
    ap.add_argument("--lens-epochs", type=int, default=300, help="training epochs of the lens-chain surrogates")
    ap.add_argument("--lens-refine", type=int, default=2,
                    help="trust-region rounds per interstage of the lens optimisation (retrain + local search)")
    ap.add_argument("--only-lens", action="store_true", help="run only the lens-optimisation study")
    ap.add_argument("--prelu-epochs", type=int, default=60,
                    help="epochs of the paper-shaped 3 x 700 surrogate trained with the paper's recipe")
    ap.add_argument("--fine-steps", type=int, default=2, help="timed steps of the fine-step path")
    ap.add_argument("--seed-sets", type=int, default=3,
                    help="init/shuffle seed sets per stage for the per-stage accuracy spread (set 0 = the chain's)")
    ap.add_argument("--only-paper-shapes", action="store_true",
                    help="run only the paper-shaped PReLU surrogate studies (inference and training)")
    ap.add_argument("--only-configs", action="store_true",
                    help="run only the timing of the other configurations (FODO, 58-element "
                         "lattice, 2000-substep stage)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline leg")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-single-stage", action="store_true",
                    help="skip the equal-error chain comparison and the single-stage (C4) study")
    ap.add_argument("--pmc-probe", action="store_true",
                    help="short run for hardware-counter passes: one plain device copy of 1 GiB "
                         "(calibration), then the benchmark's four surrogate passes (inference "
                         "with the gaps fused, untrained weights) on the benchmark bunch, twice; "
                         "with --only-configs the 58-element lattice push instead")
    return ap.parse_args()


def pmc_probe(args):
    """Short, deterministic launch sequence for rocprofv3 --pmc passes."""
    import torch

    import workloads as W
    from paper_2402_17248_amd import hbl

    from paper_2402_17248_amd.chain import Chain

    torch.cuda.set_device(0)
    a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")      # 1 GiB
    b = torch.empty_like(a)
    b.copy_(a)                                                           # reads 1 GiB, writes 1 GiB
    torch.cuda.synchronize()
    if args.only_configs:
        # the 58-element fused lattice on the benchmark bunch size, twice
        wl = W.c2_fused()
        n = args.n
        ref = hbl.Ref.from_energy(wl.E_MeV)
        lat = hbl.Lattice(wl.beamline[0], ref)
        z = hbl.new_bunch(n)
        for _ in range(2):
            hbl.fill_gaussian(z, wl.bunch.seed, (0.0,) * 6, wl.bunch.sigma, n=n)
            lat.push(z, ref.copy(), n=n)
        torch.cuda.synchronize()
        log(f"pmc probe done: copy 1 GiB, 2 x {lat.n_elem}-element lattice push on {n} particles")
        return
    wl = W.c5_chain(n=args.n)
    n = wl.bunch.n
    chain = Chain(wl.beamline, wl.E_MeV)
    sig = wl.bunch.sigma
    for k in range(chain.stage_count):
        sur = hbl.Surrogate(W.mlp_init_seed(k + 1))
        sur.set_norm([0.0] * 6 + list(sig) + [0.0] * 6 + list(sig))
        sur.set_stage(chain.stage(k), chain.entry_ref(k))
        chain.surrogates[k] = sur
    z = hbl.new_bunch(n)
    for _ in range(2):
        hbl.fill_gaussian(z, wl.bunch.seed, (0.0,) * 6, sig, n=n)
        chain.run(z, n=n, use_surrogates=True)
    torch.cuda.synchronize()
    log(f"pmc probe done: copy 1 GiB, 2 x {chain.stage_count} surrogate passes on {n} particles")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def time_events(torch, fn, iters, setup=None):
    """Average duration of fn() by HIP events on torch's current stream, the
    stream every library call below is enqueued on.  Without setup the calls
    run back to back inside one pair of events; with setup, setup() (untimed,
    enqueued first, so the device is busy while the host enqueues the call)
    runs before each separately bracketed call."""
    if setup is None:
        s = torch.cuda.Event(enable_timing=True)
        e = torch.cuda.Event(enable_timing=True)
        fn()
        s.record()
        for _ in range(iters):
            fn()
        e.record()
        torch.cuda.synchronize()
        return s.elapsed_time(e) / iters * 1e-3
    total = 0.0
    for _ in range(iters):
        setup()
        s = torch.cuda.Event(enable_timing=True)
        e = torch.cuda.Event(enable_timing=True)
        s.record()
        fn()
        e.record()
        torch.cuda.synchronize()
        total += s.elapsed_time(e)
    return total / iters * 1e-3


def host_cpu():
    """What the CPU legs ran on: the model from /proc/cpuinfo, the logical
    CPU count, the CPUs this process may run on, and the worker threads used
    (the host's share per GPU is 16 threads, whatever the machine holds)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    threads = max(1, min(16, usable))
    return {"cpu_model": model, "os_cpu_count": os.cpu_count(), "usable_cpus": usable, "threads": threads,
            "threads_note": "the GPU host grants 16 CPU threads per GPU; the pool is capped there"}


def cpu_leg(make, run, budget_s, n_max, threads, per_particle=None, min_s=0.25):
    """Time the oracle's run(z) on make(m, i0) bunches: serially on one core
    (sample sized to ~budget_s / 2), then on `threads` worker threads over
    contiguous particle ranges (threads x the serial sample, capped at
    n_max).  A run shorter than min_s is repeated on fresh copies of its
    bunch until it is not.  Bunch generation and copies are not timed.
    Returns particles/s both ways and the samples."""
    import math
    from concurrent.futures import ThreadPoolExecutor

    def timed(zs):
        t0 = time.perf_counter()
        for z in zs:
            run(z)
        return time.perf_counter() - t0

    t_small = timed([make(64, 0)]) / 64
    m1 = int(max(64, min(n_max, 0.5 * budget_s / max(t_small, 1e-12))))
    z1 = make(m1, 0)
    t1 = timed([z1.copy()])
    r1 = 1
    while t1 < min_s and r1 < 1024:        # warm repeats can run faster than the first: re-check
        r1 = min(1024, max(2 * r1, math.ceil(1.25 * min_s * r1 / max(t1, 1e-9))))
        t1 = timed([z1.copy() for _ in range(r1)])
    m2 = min(n_max, m1 * threads)
    per = (m2 + threads - 1) // threads
    with ThreadPoolExecutor(max_workers=threads) as ex:
        chunks = list(ex.map(lambda i: make(min(per, m2 - i), i), range(0, m2, per)))
        r2 = 1
        while True:
            work = [[c.copy() for _ in range(r2)] for c in chunks]
            t0 = time.perf_counter()
            list(ex.map(timed, work))
            t2 = time.perf_counter() - t0
            if t2 >= min_s or r2 >= 1024:
                break
            r2 *= 2
    out = {"serial_particles_per_s": r1 * m1 / t1, "serial_sample": m1, "serial_repeats": r1, "serial_s": t1,
           "threads_particles_per_s": r2 * m2 / t2, "threads_sample": m2, "threads_repeats": r2,
           "threads_s": t2, "threads": threads}
    if per_particle:
        for k, v in per_particle.items():
            out[f"serial_{k}_per_s"] = v * out["serial_particles_per_s"]
            out[f"threads_{k}_per_s"] = v * out["threads_particles_per_s"]
    return out


def cpu_baseline(wl, chain, budget_s):
    """The oracle, as it stands, timed on the host's cores on bounded samples
    of the same workloads (the oracle keeps no global state; ctypes releases
    the interpreter lock during its calls, so particle ranges run in parallel
    on a thread pool).  Headline leg: the staged beamline with the trained
    surrogates evaluated by the oracle's FP64 network.  Further legs: the
    fine-step staged chain (a seeded 1e6-particle subset on all threads,
    extrapolated linearly to the full bunch and labelled so), the single
    fine-step stage (C3) and one surrogate stage, the FODO cell (C1) and the
    58-element lattice (C2)."""
    import numpy as np

    import oracle
    import workloads as W

    host = host_cpu()
    T = host["threads"]
    params = [s.get_params() for s in chain.surrogates]
    norms = [np.array(s.get_norm()) for s in chain.surrogates]
    sh = oracle.shape()
    oracle.lib()

    def filler(w):
        return lambda m, i0=0: oracle.fill_gaussian(m, w.bunch.seed, (0.0,) * 6, w.bunch.sigma, i0=i0)

    def tracker(w, use_sur):
        def track(z):
            ref = oracle.Ref.from_energy(w.E_MeV)
            k = 0
            for seg in w.beamline:
                if isinstance(seg, list):
                    oracle.push(z, seg, ref)
                elif use_sur:
                    z = oracle.mlp_apply(sh, params[k], norms[k], z, mode=0)
                    ref.gamma += seg.dE_MeV / ref.mass_MeV
                    k += 1
                else:
                    oracle.push(z, [seg], ref)
            return z
        return track

    n_el = chain.n_elements()
    legs = {}
    legs["surrogate_chain_c5"] = cpu_leg(filler(wl), tracker(wl, True), budget_s, wl.bunch.n, T,
                                         {"element_pushes": n_el})
    # fine-step chain: a 1e6-particle subset on all threads, then linear
    # extrapolation to the full bunch
    sub = min(wl.bunch.n, 1_000_000)
    run_f, make_f = tracker(wl, False), filler(wl)
    z = make_f(64)
    t0 = time.perf_counter()
    run_f(z)
    m1 = int(max(64, min(sub, 0.25 * budget_s * 64 / (time.perf_counter() - t0))))
    z = make_f(m1)
    t0 = time.perf_counter()
    run_f(z)
    serial_rate = m1 / (time.perf_counter() - t0)
    from concurrent.futures import ThreadPoolExecutor
    per = (sub + T - 1) // T
    with ThreadPoolExecutor(max_workers=T) as ex:
        chunks = list(ex.map(lambda i: make_f(min(per, sub - i), i), range(0, sub, per)))
        t0 = time.perf_counter()
        list(ex.map(run_f, chunks))
        t_sub = time.perf_counter() - t0
    legs["fine_step_chain_c5"] = {
        "serial_particles_per_s": serial_rate, "serial_sample": m1,
        "threads_particles_per_s": sub / t_sub, "threads_sample": sub, "threads_s": t_sub, "threads": T,
        "full_bunch_extrapolated_threads_s": wl.bunch.n * t_sub / sub,
        "full_bunch_extrapolated_serial_s": wl.bunch.n / serial_rate,
        "note": f"measured on the first {sub} particles with {T} threads; the full-bunch times are "
                f"linear extrapolations, not measurements"}
    c3 = W.c3_stage()
    legs["fine_step_stage_c3"] = cpu_leg(filler(c3), tracker(c3, False), budget_s / 2, c3.bunch.n, T,
                                         {"substep_pushes": c3.beamline[1].nsub})
    c3_net = W.c3_stage()
    legs["surrogate_stage_fp64_network"] = cpu_leg(
        filler(c3_net), lambda z: oracle.mlp_apply(sh, params[0], norms[0], z, mode=0), budget_s / 4,
        W.C4_INFER_N, T)
    legs["surrogate_stage_fp64_network"]["note"] = ("the oracle's FP64 network (6-64-64-64-6 tanh) on "
                                                    "the C3 bunch: the cost of one surrogate stage")
    c1 = W.c1_fodo()
    legs["fodo_c1"] = cpu_leg(filler(c1), tracker(c1, False), budget_s / 8, c1.bunch.n, T,
                              {"element_pushes": len(c1.beamline[0])})
    c2 = W.c2_fused()
    legs["lattice58_c2"] = cpu_leg(filler(c2), tracker(c2, False), budget_s / 4, c2.bunch.n, T,
                                   {"element_pushes": len(c2.beamline[0])})
    head = legs["surrogate_chain_c5"]
    return {"value": head["threads_particles_per_s"], "unit": "particles/s", "cores": T, "kind": "oracle",
            "sample": f"first {head['threads_sample']} particles of the {wl.bunch.n}-particle bunch through the "
                      f"full staged beamline (lattice gaps + 4 surrogate stages, FP64 network), {T} threads "
                      f"over particle ranges, {head['threads_s']:.1f} s wall (fill excluded)",
            "serial_value": head["serial_particles_per_s"],
            "serial_sample": f"first {head['serial_sample']} particles on one core, {head['serial_s']:.1f} s",
            "host": host, "legs": legs}


def single_stage_study(args, log, chromatic=False):
    """C4: the 1 -> 10 GeV stage behind its entrance triplet.  A surrogate is
    trained on 2^20 pairs of the fine-step stage (seed 3) and applied to a
    fresh 1e7-particle bunch (seed 4); accuracy and speed against the
    2000-substep stage, and against the fine-step stage at the substep count
    whose emittance error (vs a 32,000-substep reference) equals the
    surrogate's.  chromatic: the same on the variant with chromatic triplets
    and an energy-correlated stage gain."""
    import dataclasses

    import torch

    import workloads as W
    from paper_2402_17248_amd.chain import train_concurrently
    from paper_2402_17248_amd import hbl

    wl = W.c3_chromatic() if chromatic else W.c3_stage()
    sig = wl.bunch.sigma
    stage = wl.beamline[1]

    def through_triplet(n, seed):
        z = hbl.new_bunch(n)
        hbl.fill_gaussian(z, seed, (0.0,) * 6, sig, n=n)
        ref = hbl.Ref.from_energy(wl.E_MeV)
        hbl.Lattice(wl.beamline[0], ref).push(z, ref, n=n)
        return z, ref

    npairs = W.C3_PAIR_N
    zout, ref = through_triplet(npairs, W.C3_PAIR_SEED)
    zin = hbl.new_bunch(npairs)
    entry = ref.copy()
    hbl.apply_stage(zout, stage, ref, record=zin, n=npairs)
    sur = hbl.Surrogate(W.mlp_init_seed(0))
    t0 = time.perf_counter()
    curve = sur.train(zin, zout, npairs, batch=W.TRAIN_BATCH, epochs=args.epochs, lr=W.TRAIN_LR,
                      lr_final=1e-5, train_frac=W.TRAIN_FRAC, shuffle_seed=W.shuffle_seed(0),
                      keep_best=W.TRAIN_KEEP)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    sur.set_stage(stage, entry)
    others = []                          # further init/shuffle seed sets on the same pairs, concurrently
    for sd in range(1, 1 if chromatic else args.seed_sets):
        others.append((sd, hbl.Surrogate(W.mlp_init_seed(0) + 1000 * sd)))
    train_concurrently([(o, zin, zout, npairs,
                         dict(batch=W.TRAIN_BATCH, epochs=args.epochs, lr=W.TRAIN_LR, lr_final=1e-5,
                              train_frac=W.TRAIN_FRAC, shuffle_seed=W.shuffle_seed(0) + 1000 * sd,
                              keep_best=W.TRAIN_KEEP)) for sd, o in others])
    for _, o in others:
        o.set_stage(stage, entry)
    del zin, zout

    N = W.C4_INFER_N
    x, r0 = through_triplet(N, W.C4_INFER_SEED)
    f = x.clone()
    hbl.apply_stage(f, stage, r0.copy(), n=N)
    s = x.clone()
    sur.apply(s, r0.copy(), n=N)
    rms, cen, eps = hbl.compare(s, f, n=N)
    by_seed = {"0": eps}
    for sd, o in others:
        so = x.clone()
        o.apply(so, r0.copy(), n=N)
        by_seed[str(sd)] = hbl.compare(so, f, n=N)[2]
        del so
    t_inf = time_events(torch, lambda: sur.apply(s, r0.copy(), n=N), 10)
    t_fine = time_events(torch, lambda: hbl.apply_stage(f, stage, r0.copy(), n=N), 3)
    del s, f

    # equal-error comparator on the first 1e6 particles
    m = 1_000_000
    xm = x[:, :m].contiguous()
    conv = xm.clone()
    with_nsub = lambda k: hbl.element(dataclasses.replace(stage, nsub=k))
    hbl.apply_stage(conv, with_nsub(32000), r0.copy(), n=m)
    sm = xm.clone()
    sur.apply(sm, r0.copy(), n=m)
    err_s = max(abs(e) for e in hbl.compare(sm, conv, n=m)[2][:2])

    def err_fine(nsub):
        fm = xm.clone()
        hbl.apply_stage(fm, with_nsub(nsub), r0.copy(), n=m)
        return max(abs(e) for e in hbl.compare(fm, conv, n=m)[2][:2])

    lo, hi = 50, 32000
    if err_fine(lo) <= err_s:
        hi = lo
    while hi - lo > max(1, lo // 50):
        mid = (lo + hi) // 2
        if err_fine(mid) <= err_s:
            hi = mid
        else:
            lo = mid
    n_eq = hi
    el_eq = with_nsub(n_eq)
    f2 = x.clone()
    t_fine_eq = time_events(torch, lambda: hbl.apply_stage(f2, el_eq, r0.copy(), n=N), 3)
    out = {"workload": ("stage_chromatic_1to10GeV_1e7" if chromatic else "stage_1to10GeV_1e7"),
           "particles": N, "epochs": args.epochs,
           "train_seconds": t_train, "final_loss_train_test": [float(v) for v in curve[-1]],
           "eps_rel_xyt_vs_2000_substeps": eps, "rms_over_sigma": rms, "centroid_over_sigma": cen,
           "eps_rel_xyt_by_seed_set": by_seed,
           "max_abs_eps_rel_xy_over_seed_sets": max(max(abs(v[0]), abs(v[1])) for v in by_seed.values()),
           "inference_ms": t_inf * 1e3, "fine_step_2000_ms": t_fine * 1e3, "speedup_vs_2000": t_fine / t_inf,
           "eps_err_vs_converged_32000": {"surrogate": err_s, "fine_step_at_equal_error_nsub": n_eq},
           "fine_step_equal_error_ms": t_fine_eq * 1e3, "speedup_at_equal_error": t_fine_eq / t_inf,
           "inference_particles_per_s": N / t_inf}
    log(f"{'chromatic ' if chromatic else ''}C4 single stage: eps_rel {eps}, rms {rms}; inference {t_inf*1e3:.3f} ms vs fine-step "
        f"{t_fine*1e3:.3f} ms ({t_fine/t_inf:.1f}x); equal-error fine-step nsub {n_eq} "
        f"({t_fine_eq*1e3:.3f} ms, {t_fine_eq/t_inf:.1f}x)")
    return out, t_inf


def config_studies(log):
    """Timing of the other benchmark configurations, each in the launch shape
    its parity tests use: C1 (FODO, 1e4), C2 (58-element fused lattice on
    1e6, warm and with the 256 MB last-level cache flushed, the unfused
    comparator, and 1e7 / 2.5e7 for the HBM fraction), C3 (2000-substep stage
    on 1e6)."""
    import torch

    import workloads as W
    from paper_2402_17248_amd import hbl

    out = {}
    wl = W.c1_fodo()
    n = wl.bunch.n
    z = hbl.new_bunch(n)
    hbl.fill_gaussian(z, wl.bunch.seed, (0.0,) * 6, wl.bunch.sigma, n=n)
    ref = hbl.Ref.from_energy(wl.E_MeV)
    lat = hbl.Lattice(wl.beamline[0], ref)
    t = time_events(torch, lambda: lat.push(z, ref.copy(), n=n), 50)
    out["c1_fodo_1e4"] = {"fused_us": t * 1e6, "particles_per_s": n / t,
                          "element_pushes_per_s": lat.n_elem * n / t}

    wl = W.c2_fused()
    ref = hbl.Ref.from_energy(wl.E_MeV)
    lat = hbl.Lattice(wl.beamline[0], ref)
    flush = torch.empty(1 << 27, dtype=torch.float64, device="cuda")     # 1 GiB > 256 MB cache
    c2 = {"elements": lat.n_elem}
    for n, key in ((1_000_000, "n_1e6"), (10_000_000, "n_1e7"), (25_000_000, "n_2.5e7")):
        z = hbl.new_bunch(n)
        hbl.fill_gaussian(z, wl.bunch.seed, (0.0,) * 6, wl.bunch.sigma, n=n)
        t = time_events(torch, lambda: lat.push(z, ref.copy(), n=n), 10)
        row = {"fused_us": t * 1e6, "hbm_frac": LATTICE_BYTES * n / t / (HBM_PEAK_GBS * 1e9),
               "element_pushes_per_s": lat.n_elem * n / t}
        if n == 1_000_000:
            tc = time_events(torch, lambda: lat.push(z, ref.copy(), n=n), 10, setup=lambda: flush.fill_(1.0))
            tu = time_events(torch, lambda: lat.push(z, ref.copy(), n=n, fused=False), 5)
            row.update({"fused_cold_us": tc * 1e6,
                        "hbm_frac_cold": LATTICE_BYTES * n / tc / (HBM_PEAK_GBS * 1e9),
                        "unfused_us": tu * 1e6, "fused_speedup": tu / t})
        c2[key] = row
        del z
    del flush
    out["c2_lattice58"] = c2

    wl = W.c3_stage()
    n = wl.bunch.n
    z = hbl.new_bunch(n)
    hbl.fill_gaussian(z, wl.bunch.seed, (0.0,) * 6, wl.bunch.sigma, n=n)
    ref = hbl.Ref.from_energy(wl.E_MeV)
    hbl.Lattice(wl.beamline[0], ref).push(z, ref, n=n)
    st = wl.beamline[1]
    t = time_events(torch, lambda: hbl.apply_stage(z, st, ref.copy(), n=n), 3)
    sub = st.nsub * n
    out["c3_stage_1e6"] = {"stage_ms": t * 1e3, "particles_per_s": n / t,
                           "substep_pushes_per_s": sub / t,
                           "fp64_tflops_algorithmic": 10.0 * sub / t / 1e12,
                           "fp64_flop_frac": 10.0 * sub / t / 1e12 / FP64_PEAK_TFLOPS,
                           "fp64_issue_frac": 11.0 * sub / t / (FP64_PEAK_TFLOPS / 2 * 1e12)}
    log(f"configs: C1 {out['c1_fodo_1e4']['fused_us']:.1f} us; C2 1e6 fused "
        f"{c2['n_1e6']['fused_us']:.1f} us warm / {c2['n_1e6']['fused_cold_us']:.1f} us cold, unfused "
        f"{c2['n_1e6']['unfused_us']:.1f} us, 2.5e7 {c2['n_2.5e7']['fused_us']:.0f} us "
        f"({c2['n_2.5e7']['hbm_frac']:.0%} of HBM); C3 stage {out['c3_stage_1e6']['stage_ms']:.3f} ms "
        f"({out['c3_stage_1e6']['fp64_issue_frac']:.0%} of FP64 issue)")
    return out


def lens_optimisation_study(args, log):
    """§4.4: the plasma lens of each interstage (position, focal length) is
    optimised stage by stage for the horizontal emittance after the next
    stage, with the stages taken by surrogates; the surrogate of the next
    stage is trained just before each lens is optimised, on pairs pooled over
    eight settings of that lens in the search box, then retrained around the
    lens found in each trust-region round.  The lenses found are then
    checked with the fine-step stages (full fidelity), against the starting
    lenses, and the surrogate chain's emittances against that check."""
    import workloads as W
    from paper_2402_17248_amd import hbl
    from paper_2402_17248_amd.optimize import (chain_emittances, chain_with_moment_lenses,
                                                optimise_lenses_on_surrogates)

    box = ((2.0, 7.0), (1.6, 4.0))
    wl_of = lambda lenses, n=1_000_000: W.c5_lens_chain(lenses, n=n)
    m = 1 << 17
    wl = wl_of([W.LENS_START] * 3, m)
    z0 = hbl.new_bunch(m)
    hbl.fill_gaussian(z0, wl.bunch.seed, (0.0,) * 6, wl.bunch.sigma, n=m)
    stages = [hbl.element(seg) for seg in wl.beamline if not isinstance(seg, list)]

    def apply_fine(k, z, ref, pre, n):
        hbl.apply_stage(z, stages[k], ref, n=n, pre=pre)

    t0 = time.perf_counter()
    lenses, eps_opt, report, surs, training_sets, t_train = optimise_lenses_on_surrogates(
        wl_of, W.LENS_START, z0, m, box, 1 << 20, args.lens_epochs, lambda k: 300 + k,
        lambda k: W.mlp_init_seed(k + 1), lambda k: W.shuffle_seed(k + 1),
        refine_rounds=args.lens_refine, log=log)
    t_opt = time.perf_counter() - t0 - t_train
    evals = sum(r["evaluations"] for r in report)

    def apply_sur(k, z, ref, pre, n):
        surs[k].apply(z, ref, n=n, pre=pre)

    N = 1_000_000
    zf = hbl.new_bunch(N)
    hbl.fill_gaussian(zf, 55, (0.0,) * 6, wl.bunch.sigma, n=N)
    bg = [math.sqrt(((1000.0 + 10000.0 * (k + 1)) / hbl.MEC2_MEV) ** 2 - 1) for k in range(4)]
    norm = lambda e: [v * b for v, b in zip(e, bg)]
    fine_start = norm(chain_emittances(wl_of([W.LENS_START] * 3, N), zf, N, apply_fine))
    fine_opt = norm(chain_emittances(wl_of(lenses, N), zf, N, apply_fine))
    sur_opt = norm(chain_emittances(wl_of(lenses, N), zf, N, apply_sur))
    # the paper's reference strategy: centred lenses set from the moments after each stage
    mom_lenses, mom_eps = chain_with_moment_lenses(lambda L: wl_of(L, N), zf, N, apply_fine,
                                                   W.LENS_GAP_LENGTH / 2)
    fine_mom = norm(mom_eps)
    log(f"lens optimisation: {evals} surrogate-chain evaluations in {t_opt:.2f} s "
        f"({evals / t_opt:.0f}/s on {m} particles); normalised eps_x after stages 1-4, fine-step "
        f"check: start {['%.3e' % v for v in fine_start]}, optimised {['%.3e' % v for v in fine_opt]} "
        f"(surrogate chain {['%.3e' % v for v in sur_opt]}); moment-driven centred lenses "
        f"{['%.3e' % v for v in fine_mom]}")
    return {"lenses_start": [W.LENS_START] * 3, "lenses_found": lenses, "training_seconds": t_train,
            "training_lens_settings": training_sets, "evaluations": evals, "optimisation_seconds": t_opt,
            "evaluations_per_s": evals / t_opt, "sample_particles": m, "check_particles": N,
            "eps_nx_fine_step_start": fine_start, "eps_nx_fine_step_optimised": fine_opt,
            "eps_nx_surrogate_optimised": sur_opt,
            "surrogate_prediction_rel_error": [a / b - 1 for a, b in zip(sur_opt, fine_opt)],
            "refine_rounds": args.lens_refine, "per_interstage": report,
            "moment_driven_lenses": mom_lenses, "eps_nx_fine_step_moment_driven": fine_mom}


# §4.3: inference of 1e7 particles on one A100 took 1.12 s per stage for the
# 5 x 900 networks (stages 1-3) and 494 ms for the 3 x 700 ones (stages 4-15),
# 63.2 ns per particle and stage averaged over the 15 stages.
PAPER_A100_S_PER_1E7 = {(900, 5): 1.12, (700, 3): 0.494}
PAPER_A100_NS_AVG = 63.2
# §4.2: batch 1200, learning rate 1e-4, 1500 epochs; about 2.2 h per stage
# (5 x 900) and 2 h (3 x 700) on one A100.
PAPER_BATCH, PAPER_LR, PAPER_EPOCHS = 1200, 1e-4, 1500
PAPER_A100_TRAIN_H = {(900, 5): 2.2, (700, 3): 2.0}


def paper_shape_training(args, log):
    """Train the paper-shaped networks with the paper's recipe on the C4
    stage pairs (2^20 pairs of the fine-step stage behind its triplet), then
    apply the trained 3 x 700 network to the 1e7-particle C4 bunch and
    compare with the 2000-substep stage."""
    import torch

    import workloads as W
    from paper_2402_17248_amd import hbl

    wl = W.c3_stage()
    sig, stage = wl.bunch.sigma, wl.beamline[1]

    def through_triplet(n, seed):
        z = hbl.new_bunch(n)
        hbl.fill_gaussian(z, seed, (0.0,) * 6, sig, n=n)
        ref = hbl.Ref.from_energy(wl.E_MeV)
        hbl.Lattice(wl.beamline[0], ref).push(z, ref, n=n)
        return z, ref

    npairs = W.C3_PAIR_N
    zout, ref = through_triplet(npairs, W.C3_PAIR_SEED)
    zin = hbl.new_bunch(npairs)
    entry = ref.copy()
    hbl.apply_stage(zout, stage, ref, record=zin, n=npairs)
    n_train, _ = W.split_counts(npairs)
    out = {}
    trained = None
    for (width, hidden), epochs in (((700, 3), args.prelu_epochs), ((900, 5), 2)):
        net = hbl.PreluNet(width, hidden, W.mlp_init_seed(0))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        curve = net.train(zin, zout, npairs, batch=PAPER_BATCH, epochs=epochs, lr=PAPER_LR, lr_final=PAPER_LR / 10,
                          train_frac=W.TRAIN_FRAC, shuffle_seed=W.shuffle_seed(0))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        steps = epochs * (n_train // PAPER_BATCH)
        per_epoch = dt / epochs
        out[f"{hidden}x{width}"] = {
            "epochs": epochs, "seconds": dt, "seconds_per_epoch": per_epoch,
            "samples_per_s": steps * PAPER_BATCH / dt, "us_per_step_incl_test_loss": dt / steps * 1e6,
            "final_loss_train_test": [float(v) for v in curve[-1]],
            "projected_1500_epochs_s": per_epoch * PAPER_EPOCHS,
            "paper_a100_hours_1500_epochs": PAPER_A100_TRAIN_H[(width, hidden)]}
        if (width, hidden) == (700, 3):
            trained = net
        else:
            net.close()
    del zin, zout
    trained.set_stage(stage, entry)
    N = W.C4_INFER_N
    x, r0 = through_triplet(N, W.C4_INFER_SEED)
    f = x.clone()
    hbl.apply_stage(f, stage, r0.copy(), n=N)
    x_s = x.clone()
    trained.apply(x_s, r0.copy(), n=N)
    rms, cen, eps = hbl.compare(x_s, f, n=N)
    out["3x700"]["c4_eps_rel_xyt_vs_2000_substeps"] = eps
    out["3x700"]["c4_rms_over_sigma"] = rms
    log(f"paper-recipe training: 3x700 {out['3x700']['epochs']} epochs in {out['3x700']['seconds']:.1f} s "
        f"({out['3x700']['samples_per_s']:.3g} samples/s; 1500 epochs ~{out['3x700']['projected_1500_epochs_s']:.0f} s, "
        f"paper A100 ~2 h), final loss {out['3x700']['final_loss_train_test']}; 5x900 "
        f"{out['5x900']['seconds_per_epoch']:.2f} s/epoch; trained 3x700 on C4 1e7: eps_rel {eps}, rms {rms}")
    return out


def paper_shape_chain(args, log, wl, time_chain, dt_fine, z_fine):
    """The staged chain with the paper's own networks: one 3 x 700 PReLU
    surrogate per stage, trained with the paper's recipe on that stage's
    pairs, run on the same 2.5e7-particle bunch as the headline chain."""
    import torch

    import workloads as W
    from paper_2402_17248_amd import hbl
    from paper_2402_17248_amd.chain import Chain, train_concurrently

    c = Chain(wl.beamline, wl.E_MeV)
    n = wl.bunch.n
    t0 = time.perf_counter()
    # the four stages' networks trained at the same time, each on its own stream
    pairs = [c.make_pairs(k, args.pairs, W.c5_pair_seed(k + 1), wl.bunch.sigma) for k in range(c.stage_count)]
    nets = [hbl.PreluNet(700, 3, W.mlp_init_seed(k + 1)) for k in range(c.stage_count)]
    curves = train_concurrently([(nets[k], *pairs[k], args.pairs,
                                  dict(batch=PAPER_BATCH, epochs=args.prelu_epochs // 2, lr=PAPER_LR,
                                       lr_final=PAPER_LR / 10, train_frac=W.TRAIN_FRAC,
                                       shuffle_seed=W.shuffle_seed(k + 1))) for k in range(c.stage_count)])
    del pairs
    losses = []
    for k, (net, curve) in enumerate(zip(nets, curves)):
        net.set_stage(c.stage(k), c.entry_ref(k))
        c.surrogates[k] = net
        losses.append([float(v) for v in curve[-1]])
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    dt = time_chain(lambda zz: c.run(zz, n=n, use_surrogates=True), 3, 1)
    zs = hbl.new_bunch(n)
    hbl.fill_gaussian(zs, wl.bunch.seed, (0.0,) * 6, wl.bunch.sigma, n=n)
    c.run(zs, n=n, use_surrogates=True)
    rms, cen, eps = hbl.compare(zs, z_fine, n=n)
    del zs
    out = {"network": "PReLU 6-700-700-700-6 per stage", "epochs_per_stage": args.prelu_epochs // 2,
           "train_seconds": t_train, "final_loss_train_test": losses, "ms_per_step": dt * 1e3,
           "particles_per_s": n / dt, "speedup_vs_fine_step_chain": dt_fine / dt,
           "eps_rel_xyt_vs_fine_step_chain": eps, "rms_over_sigma": rms}
    log(f"chain with paper-shaped surrogates: {dt * 1e3:.1f} ms/step ({n / dt:.3g} particles/s, "
        f"{dt_fine / dt:.1f}x the fine-step chain); eps_rel vs fine-step chain {eps}; trained in {t_train:.1f} s")
    for sur in c.surrogates:
        sur.close()
    return out


def paper_shape_study(log):
    """The paper's own network shapes (PReLU, 5 x 900 and 3 x 700) on the C4
    inference workload (1e7 particles): inference time, dense-layer rate on
    the matrix cores, and the 15-stage average the paper quotes."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2402_17248_amd import hbl

    N = W.C4_INFER_N
    wl = W.c3_stage(n=8)
    sd = np.asarray(wl.bunch.sigma)
    norm = np.concatenate([0.0 * sd, sd, 0.0 * sd, sd])
    z = hbl.new_bunch(N)
    out = {}
    for width, hidden in ((900, 5), (700, 3)):
        net = hbl.PreluNet(width, hidden, W.mlp_init_seed(0))
        net.set_norm(norm)
        hbl.fill_gaussian(z, W.C4_INFER_SEED, (0.0,) * 6, wl.bunch.sigma, n=N)
        t = time_events(torch, lambda: net.apply(z, n=N), 5)
        fl = net.flops_per_particle()
        tflops = fl * N / t / 1e12
        out[f"{hidden}x{width}"] = {
            "ms_per_1e7": t * 1e3, "ns_per_particle": t / N * 1e9, "flop_per_particle": fl,
            "dense_tflops": tflops, "mfma_frac": tflops / BF16_PEAK_TFLOPS,
            "paper_a100_ms_per_1e7": PAPER_A100_S_PER_1E7[(width, hidden)] * 1e3,
            "ratio_to_paper_a100": PAPER_A100_S_PER_1E7[(width, hidden)] / t}
        net.close()
    avg = (3 * out["5x900"]["ns_per_particle"] + 12 * out["3x700"]["ns_per_particle"]) / 15
    out["avg_15_stages_ns_per_particle"] = avg
    out["paper_a100_avg_ns_per_particle"] = PAPER_A100_NS_AVG
    log(f"paper-shaped PReLU surrogates on 1e7 particles: 5x900 {out['5x900']['ms_per_1e7']:.1f} ms "
        f"({out['5x900']['dense_tflops']:.0f} TFLOP/s, {out['5x900']['mfma_frac']:.0%} of MFMA peak), "
        f"3x700 {out['3x700']['ms_per_1e7']:.1f} ms ({out['3x700']['dense_tflops']:.0f} TFLOP/s); "
        f"15-stage average {avg:.2f} ns/particle/stage (paper, A100: {PAPER_A100_NS_AVG} ns)")
    return out


def stage_accuracy_study(args, log, wl, chain):
    """Each chain stage's surrogate against its own fine-step map on the
    chain's own inputs: the full bunch tracked with fine-step stages to the
    stage entrance, then the stage (fine-step) and the surrogate applied to
    the same particles.  The networks of the chain (seed set 0) and networks
    trained with further init/shuffle seed sets on the same pairs give the
    spread of the per-stage emittance error over seeds."""
    import workloads as W
    from paper_2402_17248_amd import hbl

    from paper_2402_17248_amd.chain import train_concurrently

    n, sig = wl.bunch.n, wl.bunch.sigma
    seeds = list(range(args.seed_sets))
    # the further seed sets' networks of every stage, trained at the same time
    extra, jobs, pairs = {}, [], {}
    for k in range(chain.stage_count if len(seeds) > 1 else 0):
        pairs[k] = chain.make_pairs(k, args.pairs, W.c5_pair_seed(k + 1), sig)
        for sd in seeds[1:]:
            extra[(k, sd)] = hbl.Surrogate(W.mlp_init_seed(k + 1) + 1000 * sd)
            jobs.append((extra[(k, sd)], *pairs[k], args.pairs,
                         dict(batch=W.TRAIN_BATCH, epochs=args.epochs, lr=W.TRAIN_LR, lr_final=1e-5,
                              train_frac=W.TRAIN_FRAC, shuffle_seed=W.shuffle_seed(k + 1) + 1000 * sd,
                              keep_best=W.TRAIN_KEEP)))
    t0 = time.perf_counter()
    train_concurrently(jobs)
    if jobs:
        log(f"seed-set networks: {len(jobs)} trained concurrently in {time.perf_counter() - t0:.1f} s")
    del jobs, pairs
    out = []
    for k in range(chain.stage_count):
        zin, zout = chain.make_pairs(k, n, wl.bunch.seed, sig)
        stage, entry = chain.stage(k), chain.entry_ref(k)
        nets = {0: chain.surrogates[k]}
        for sd in seeds[1:]:
            extra[(k, sd)].set_stage(stage, entry)
            nets[sd] = extra[(k, sd)]
        row = {"stage": k + 1, "particles": n, "by_seed_set": {}}
        for sd, sur in nets.items():
            zs = zin.clone()
            sur.apply(zs, entry.copy(), n=n)
            rms, cen, eps = hbl.compare(zs, zout, n=n)
            del zs
            row["by_seed_set"][str(sd)] = {"eps_rel_xyt": eps, "rms_over_sigma": rms, "centroid_over_sigma": cen}
        worst = max(max(abs(v["eps_rel_xyt"][0]), abs(v["eps_rel_xyt"][1])) for v in row["by_seed_set"].values())
        row["max_abs_eps_rel_xy_over_seed_sets"] = worst
        log(f"stage {k + 1} surrogate vs its fine-step map on the chain's inputs: eps_rel x,y by seed set "
            + ", ".join(f"{sd}: [{v['eps_rel_xyt'][0]:+.2e}, {v['eps_rel_xyt'][1]:+.2e}]"
                        for sd, v in row["by_seed_set"].items()))
        out.append(row)
        del zin, zout, nets
    return out


def chain_equal_error(args, wl, chain, dt_sur, step_fn, log):
    """The staged chain at equal error: on the first 1e6 particles of the
    benchmark bunch, the emittance error of the surrogate chain and of the
    fine-step chain at a given substep count are measured against the
    fine-step chain at 32,000 substeps per stage; the substep count whose
    error equals the surrogate chain's is found by bisection and that
    fine-step chain is timed on the full bunch like the benchmark step."""
    import torch

    import workloads as W
    from paper_2402_17248_amd import hbl
    from paper_2402_17248_amd.chain import Chain

    m = 1_000_000
    sig = wl.bunch.sigma
    z0 = hbl.new_bunch(m)
    hbl.fill_gaussian(z0, wl.bunch.seed, (0.0,) * 6, sig, n=m)

    def fine(nsub, n, z):
        c = Chain(W.c5_chain(n=n, nsub=nsub).beamline, wl.E_MeV)
        c.run(z, n=n)
        return c

    conv = z0.clone()
    fine(32000, m, conv)
    zs = z0.clone()
    chain.run(zs, n=m, use_surrogates=True)
    err_s = max(abs(e) for e in hbl.compare(zs, conv, n=m)[2][:2])

    def err_fine(nsub):
        zf = z0.clone()
        fine(nsub, m, zf)
        return max(abs(e) for e in hbl.compare(zf, conv, n=m)[2][:2])

    err_2000 = err_fine(wl.beamline[1].nsub)
    lo, hi = 50, 32000
    if err_fine(lo) <= err_s:
        hi = lo
    while hi - lo > max(1, lo // 50):
        mid = (lo + hi) // 2
        if err_fine(mid) <= err_s:
            hi = mid
        else:
            lo = mid
    n_eq = hi
    del z0, conv, zs
    eq_chain = Chain(W.c5_chain(n=wl.bunch.n, nsub=n_eq).beamline, wl.E_MeV)
    dt_eq = step_fn(eq_chain, 2, 1)
    n = wl.bunch.n
    log(f"chain at equal error: surrogate emittance error {err_s:.3e} vs 32000-substep chain "
        f"(2000 substeps: {err_2000:.3e}); fine-step chain needs {n_eq} substeps per stage: "
        f"{dt_eq * 1e3:.3f} ms/step, surrogate chain {dt_eq / dt_sur:.1f}x faster")
    return {"eps_err_vs_32000_substep_chain": {"surrogate": err_s, "fine_step_2000": err_2000},
            "fine_step_equal_error_nsub": n_eq, "fine_step_equal_error_ms_per_step": dt_eq * 1e3,
            "fine_step_equal_error_particles_per_s": n / dt_eq, "speedup_at_equal_error": dt_eq / dt_sur}


def main():
    args = parse()
    if args.pmc_probe:
        pmc_probe(args)
        return
    if args.only_configs:
        import torch
        torch.cuda.set_device(0)
        print(json.dumps({"other_configs": config_studies(log)}), flush=True)
        return
    if args.only_lens:
        import torch
        torch.cuda.set_device(0)
        print(json.dumps({"lens_optimisation": lens_optimisation_study(args, log)}), flush=True)
        return
    if args.only_paper_shapes:
        import torch
        torch.cuda.set_device(0)
        out = paper_shape_study(log)
        out["training"] = paper_shape_training(args, log)
        print(json.dumps({"paper_shaped_surrogates": out}), flush=True)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU only; there is no multi-GPU path "
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
                                    keep_best=W.TRAIN_KEEP,
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

    n_pass = len(chain.passes())        # stage passes per step, one kernel launch each

    def step(use_sur, ev=None):
        if ev is not None:
            ev[0].record()
        hbl.fill_gaussian(z, wl.bunch.seed, (0.0,) * 6, sig, n=n)
        if ev is not None:
            ev[1].record()
        chain.run(z, n=n, use_surrogates=use_sur)
        if ev is not None:
            ev[2].record()
        hbl.moments_async(z, out27, n=n)
        if ev is not None:
            ev[3].record()

    breakdown = {}

    def timed(use_sur, steps, warmup):
        """Wall time per step over exactly `steps` steps, and the average
        duration of one stage-pass launch from HIP events recorded on the
        library's stream around the passes inside those same steps (events
        around the fill and the moments give the rest of the step)."""
        for _ in range(warmup):
            step(use_sur)
        evs = [tuple(torch.cuda.Event(enable_timing=True) for _ in range(4)) for _ in range(steps)]
        torch.cuda.synchronize()
        t = time.perf_counter()
        for k in range(steps):
            step(use_sur, evs[k])
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t) / steps
        part = [sum(e[j].elapsed_time(e[j + 1]) for e in evs) / steps for j in range(3)]
        breakdown["surrogate" if use_sur else "fine_step"] = {
            "fill_ms": part[0], "stage_passes_ms": part[1], "moments_ms": part[2]}
        per_launch = part[1] * 1e-3 / n_pass
        return dt, per_launch

    def time_chain(c, steps, warmup):
        """c: a Chain (run with its fine-step stages) or a callable run(z)."""
        def one():
            hbl.fill_gaussian(z, wl.bunch.seed, (0.0,) * 6, sig, n=n)
            if callable(c):
                c(z)
            else:
                c.run(z, n=n)
            hbl.moments_async(z, out27, n=n)
        for _ in range(warmup):
            one()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            one()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / steps

    dt_sur, t_inf = timed(True, args.steps, args.warmup)
    log(f"surrogate chain: {dt_sur * 1e3:.3f} ms/step, {n / dt_sur:.4g} particles/s (HIP events: fill "
        f"{breakdown['surrogate']['fill_ms']:.3f} ms, {n_pass} stage passes "
        f"{breakdown['surrogate']['stage_passes_ms']:.3f} ms, moments {breakdown['surrogate']['moments_ms']:.3f} ms)")
    dt_fine, t_fs = timed(False, args.fine_steps, 1)
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
    z_fine = z.clone()                  # the fine-step chain's result, kept for the paper-shaped chain

    equal = configs = per_stage = None
    if not args.no_single_stage:
        per_stage = stage_accuracy_study(args, log, wl, chain)
        equal = chain_equal_error(args, wl, chain, dt_sur, time_chain, log)
        configs = config_studies(log)

    single = single_chrom = lens_opt = paper_shapes = None
    if not args.no_single_stage:
        single, _ = single_stage_study(args, log)
        single_chrom, _ = single_stage_study(args, log, chromatic=True)
        lens_opt = lens_optimisation_study(args, log)
        paper_shapes = paper_shape_study(log)
        paper_shapes["training"] = paper_shape_training(args, log)
        paper_shapes["chain"] = paper_shape_chain(args, log, wl, time_chain, dt_fine, z_fine)
    del z_fine

    # ---- dominant kernel: surrogate inference with the gaps fused (k_mlp_infer,
    # one launch per stage pass), timed inside the timed steps above
    alu_achieved = ALU_SLOTS_PER_PARTICLE * n / t_inf / 1e12
    mfma_achieved = MLP_FLOP_PER_PARTICLE * n / t_inf / 1e12
    log(f"inference kernel (gaps fused): {t_inf * 1e3:.3f} ms per launch ({n / t_inf:.4g} particles/s, "
        f"{alu_achieved:.1f} T VALU slots/s, {mfma_achieved:.0f} TFLOP/s dense); fine-step stage "
        f"kernel: {t_fs * 1e3:.3f} ms per launch; per-stage speed-up {t_fs / t_inf:.1f}x")

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(wl, chain, args.cpu_seconds)
        log(f"cpu oracle: {cpu['value']:.4g} particles/s ({cpu['sample']}); host {cpu['host']}")
        for k, v in cpu["legs"].items():
            log(f"cpu oracle leg {k}: serial {v['serial_particles_per_s']:.4g}, {v['threads']} threads "
                f"{v['threads_particles_per_s']:.4g} particles/s")

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
        "fine_step_path": {"value": n / dt_fine, "ms_per_step": dt_fine * 1e3, "nsub": chain.stage(0).nsub,
                           "speedup_surrogate": dt_fine / dt_sur},
        "accuracy_vs_fine_step": {"eps_rel_xyt": eps_rel, "rms_over_sigma": rms,
                                  "centroid_over_sigma": cen, "per_stage": per_stage},
        "step_breakdown_ms": breakdown,
        "stage_pass_kernels": {"inference_ms": t_inf * 1e3, "fine_step_ms": t_fs * 1e3,
                               "speedup": t_fs / t_inf, "launches_per_step": n_pass,
                               "dense_mfma_tflops": mfma_achieved,
                               "dense_mfma_frac": mfma_achieved / BF16_PEAK_TFLOPS},
        "chain_equal_error": equal,
        "other_configs": configs,
        "single_stage_c4": single,
        "single_stage_c4_chromatic": single_chrom,
        "lens_optimisation": lens_opt,
        "paper_shaped_surrogates": paper_shapes,
        "particle_element_pushes_per_s": chain.n_elements() * n / dt_sur,
        "roofline": {"bound": "alu", "achieved": alu_achieved, "peak": VALU_PEAK_TSLOTS,
                     "unit": "T VALU slots/s", "frac": alu_achieved / VALU_PEAK_TSLOTS,
                     "traffic": TRAFFIC_BYTES_PER_LAUNCH if n == 25_000_000 else None,
                     "traffic_unit": "HBM bytes per launch (algorithmic 96 B/particle)",
                     "kernel": "k_mlp_infer<gaps> (surrogate inference, transport gaps fused)"},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
