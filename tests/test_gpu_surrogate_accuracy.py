"""What the trained network gains over the method without it (§1: a stage
as a transfer map; the traditional map is linear).  A surrogate trained on the
GPU by the library's own kernels is compared, on a fresh bunch, with the
affine least-squares transfer map fitted to the same training pairs, both
against the fine-step stage.  The bounds are loose on purpose (a quarter of the
benchmark's pairs); the benchmark reports the full-length numbers."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def test_network_beats_linear_transfer_map():
    import torch

    from paper_2402_17248_amd import hbl
    n_pairs = 1 << 18
    wl = W.c3_stage()
    sig = wl.bunch.sigma

    def through_triplet(n, seed):
        z = hbl.new_bunch(n)
        hbl.fill_gaussian(z, seed, (0.0,) * 6, sig, n=n)
        ref = hbl.Ref.from_energy(wl.E_MeV)
        hbl.Lattice(wl.beamline[0], ref).push(z, ref, n=n)
        return z, ref

    zout, ref = through_triplet(n_pairs, W.C3_PAIR_SEED)
    zin = hbl.new_bunch(n_pairs)
    entry = ref.copy()
    hbl.apply_stage(zout, wl.beamline[1], ref, record=zin, n=n_pairs)
    sur = hbl.Surrogate(W.mlp_init_seed(1))
    log = sur.train(zin, zout, n_pairs, batch=4096, epochs=300, lr=1e-3, lr_final=1e-5,
                    shuffle_seed=W.shuffle_seed(1))
    assert log[-1, 1] < 0.05 * log[0, 1]          # test loss fell by > 20x

    n = 1_000_000
    x, r0 = through_triplet(n, W.C4_INFER_SEED)
    f = x.clone()
    hbl.apply_stage(f, wl.beamline[1], r0.copy(), n=n)
    s = x.clone()
    sur.set_stage(wl.beamline[1], entry)
    rs = r0.copy()
    sur.apply(s, rs, n=n)
    rms_nn, _, eps_nn = hbl.compare(s, f, n=n)

    # affine transfer map y = M [x; 1], least squares on the training pairs
    X = zin[:, :n_pairs].double().cpu().numpy().T
    Y = zout[:, :n_pairs].double().cpu().numpy().T
    M, *_ = np.linalg.lstsq(np.hstack([X, np.ones((n_pairs, 1))]), Y, rcond=None)
    xi = x[:, :n].cpu().numpy().T
    lin = torch.from_numpy(np.ascontiguousarray((np.hstack([xi, np.ones((n, 1))]) @ M).T)).cuda()
    zl = hbl.new_bunch(n)
    zl[:, :n] = lin
    rms_lin, _, eps_lin = hbl.compare(zl, f, n=n)

    assert max(abs(eps_nn[0]), abs(eps_nn[1])) < 2e-2, eps_nn
    assert min(abs(eps_lin[0]), abs(eps_lin[1])) > 0.5, eps_lin   # the linear map misses the filamentation
    assert max(rms_nn[:2]) < 0.1 * min(rms_lin[:2]), (rms_nn, rms_lin)
