"""The moments call that allocates nothing (hbl_moments_async_noalloc),
through the C ABI: on two calls in a row, the second with a smaller bunch,
its 27 values equal those of hbl_moments_async on the same bunch bit for bit
(same kernels and grid; only the scratch differs), and both lie within the
reductions' parity bar (1e-13) of the oracle's exact moments of the same
bytes (bunches made by the oracle and uploaded)."""
import ctypes as C

import numpy as np
import pytest

import workloads as W
from gpu_util import to_dev

pytestmark = pytest.mark.gpu


def _exact_errors(orc, out, host):
    om, oc = orc.moments(host)
    Co = orc.cov_matrix(oc)
    Cg = orc.cov_matrix(out[6:])
    sd = np.sqrt(np.diag(Co))
    em = np.abs((out[:6] - om) / np.maximum(sd, np.abs(om))).max()
    ec = np.abs((Cg - Co) / np.outer(sd, sd)).max()
    return em, ec


def test_noalloc_moments_match_allocating_call(orc):
    import torch

    from paper_2402_17248_amd import hbl

    lib = hbl.lib
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    sig = W.BunchSpec(1, 1).sigma
    # the first bunch spans the full 1024-block grid and has a ragged tail;
    # the second is smaller and offset, so stale partials of the first call
    # would show
    for n, seed, shift in ((1_000_003, 21, 0.0), (4_097, 22, 3.0)):
        print(f"noalloc moments: n={n} seed={seed}", flush=True)
        host = orc.fill_gaussian(n, seed, tuple(shift * s for s in sig), sig)
        z = to_dev(host)
        ld = z.shape[1]
        a = torch.full((27,), float("nan"), dtype=torch.float64, device="cuda")
        b = torch.full((27,), float("nan"), dtype=torch.float64, device="cuda")
        rc = lib.hbl_moments_async_noalloc(C.c_void_p(z.data_ptr()), n, ld, C.c_void_p(a.data_ptr()), stream)
        assert rc == 0, lib.hbl_last_error().decode()
        rc = lib.hbl_moments_async(C.c_void_p(z.data_ptr()), n, ld, C.c_void_p(b.data_ptr()), stream)
        assert rc == 0, lib.hbl_last_error().decode()
        torch.cuda.synchronize()
        ga, gb = a.cpu().numpy(), b.cpu().numpy()
        assert np.array_equal(ga, gb), np.abs(ga - gb).max()
        em, ec = _exact_errors(orc, ga, host)
        print(f"  bitwise equal to hbl_moments_async; vs exact: mean {em:.2e}, cov {ec:.2e}", flush=True)
        assert em < 1e-13 and ec < 1e-13, (em, ec)
