"""Accuracy of the trained surrogate against the fine-step stage.

* The accuracy bar: the 1 -> 10 GeV stage behind its entrance triplet,
  trained with the benchmark's recipe (2^20 pairs of the fine-step stage,
  batch 4096, 1200 epochs, lr 1e-3 annealed by a half cosine to 1e-5, model
  selection on the 30 % test split: among the last quarter of the epochs
  with a test loss within 10 % of the lowest, the one whose test-split
  emittances are closest to the true ones), is applied to a fresh bunch of
  1e7 particles; its emittances in x and y lie within 1e-3 of those of the
  2000-substep stage on the same bunch.  The emittance error of a trained
  network is seed dependent (the benchmark reports its spread over seeds);
  this test pins the benchmark's own seeds, a deterministic pipeline.
* What the trained network gains over the method without it (§1: a stage
  as a transfer map; the traditional map is linear): a surrogate trained on
  a quarter of the pairs for 300 epochs is compared, on a fresh bunch, with
  the affine least-squares transfer map fitted to the same training pairs,
  both against the fine-step stage."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def test_accuracy_bar_single_stage():
    import torch

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
    sur = hbl.Surrogate(W.mlp_init_seed(0))
    log = sur.train(zin, zout, npairs, batch=W.TRAIN_BATCH, epochs=1200, lr=W.TRAIN_LR, lr_final=1e-5,
                    train_frac=W.TRAIN_FRAC, shuffle_seed=W.shuffle_seed(0), keep_best=W.TRAIN_KEEP)
    sur.set_stage(stage, entry)
    del zin, zout
    n = W.C4_INFER_N
    x, r0 = through_triplet(n, W.C4_INFER_SEED)
    f = x.clone()
    hbl.apply_stage(f, stage, r0.copy(), n=n)
    sur.apply(x, r0.copy(), n=n)
    rms, cen, eps = hbl.compare(x, f, n=n)
    torch.cuda.synchronize()
    print(f"C4 stage, benchmark recipe: lowest test loss {log[:, 1].min():.3e} after epoch "
          f"{int(log[:, 1].argmin())}; eps_s/eps_f - 1 (x, y, t) = {eps}; rms/sigma = {rms}", flush=True)
    assert abs(eps[0]) <= 1e-3 and abs(eps[1]) <= 1e-3, eps
    assert max(rms) < 5e-3, rms


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
                    shuffle_seed=W.shuffle_seed(1), keep_best=W.TRAIN_KEEP)
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

    print(f"network vs fine-step: eps {eps_nn}, rms {rms_nn}; affine map: eps {eps_lin}, rms {rms_lin}", flush=True)
    assert max(abs(eps_nn[0]), abs(eps_nn[1])) < 1e-2, eps_nn
    assert min(abs(eps_lin[0]), abs(eps_lin[1])) > 0.5, eps_lin   # the linear map misses the filamentation
    assert max(rms_nn[:2]) < 0.1 * min(rms_lin[:2]), (rms_nn, rms_lin)
