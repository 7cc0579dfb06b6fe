"""Host-side parts of the benchmark that run without a GPU: the CPU
baseline's host description and its timing legs (the oracle on bounded
samples, serially and on a thread pool)."""
import numpy as np

import bench


def test_host_cpu_description():
    h = bench.host_cpu()
    assert h["cpu_model"] and h["os_cpu_count"] >= 1
    assert 1 <= h["threads"] <= 16 and h["threads"] <= h["usable_cpus"]


def test_cpu_leg_times_serial_and_threads(orc):
    import workloads as W
    wl = W.c1_fodo()
    make = lambda m, i0=0: orc.fill_gaussian(m, wl.bunch.seed, (0.0,) * 6, wl.bunch.sigma, i0=i0)
    run = lambda z: orc.push(z, wl.beamline[0], orc.Ref.from_energy(wl.E_MeV))
    out = bench.cpu_leg(make, run, 0.2, wl.bunch.n, 2, {"element_pushes": 5}, min_s=0.05)
    assert out["serial_sample"] <= wl.bunch.n and out["threads_sample"] <= wl.bunch.n
    assert out["serial_particles_per_s"] > 0 and out["threads_particles_per_s"] > 0
    assert out["serial_s"] >= 0.05 and out["threads_s"] >= 0.05        # short runs were repeated
    assert np.isclose(out["serial_element_pushes_per_s"], 5 * out["serial_particles_per_s"])
