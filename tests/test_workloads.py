"""The benchmark beamline's own design property, checked with the oracle's
element maps: each interstage of the staged chain (§4, Fig. 1: stages joined
by transport) images the exit of one stage onto the entrance of the next,
point to point in both planes with magnification -1, so a beam that leaves a
stage matched enters the next one matched."""
import numpy as np

import workloads as W


def transfer_matrix(orc, elems, E_MeV):
    z = np.ascontiguousarray(np.eye(6))
    orc.push(z, elems, orc.Ref.from_energy(E_MeV))
    return z          # column j = image of unit vector j


def test_interstage_images_point_to_point(orc):
    for E in (11_000.0, 21_000.0, 31_000.0):
        R = transfer_matrix(orc, W.interstage(), E)
        assert abs(R[0, 3]) < 1e-8 and abs(R[1, 4]) < 1e-8          # R12, R34 (m)
        assert abs(R[0, 0] + 1) < 1e-3 and abs(R[1, 1] + 1) < 1e-3  # R11, R33
        assert abs(R[3, 3] + 1) < 1e-3 and abs(R[4, 4] + 1) < 1e-3  # R22, R44
        assert abs(R[0, 5]) < 1e-5                                   # residual dispersion (m)
    assert len(W.interstage()) == 15
    assert abs(sum(e.L for e in W.interstage()) - 13.3) < 1e-12


def test_chain_keeps_the_beam_bounded(orc):
    """Through four stages the transverse size stays within a factor 3 of the
    first stage's exit, and the normalised emittance grows by < 50 % after the
    first (mismatched) stage."""
    wl = W.c5_chain(n=2000, nsub=500)
    c = orc.fill_gaussian(2000, 5, (0.0,) * 6, wl.bunch.sigma)
    ref = orc.Ref.from_energy(wl.E_MeV)
    sizes, eps_n = [], []
    for seg in wl.beamline[:-1]:
        orc.push(c, seg if isinstance(seg, list) else [seg], ref)
        if not isinstance(seg, list):
            _, cov = orc.moments(c)
            sizes.append(np.sqrt(cov[0]))
            bg = np.sqrt(ref.gamma ** 2 - 1)
            eps_n.append(bg * orc.emittances(cov)[0])
    assert max(sizes) < 3 * sizes[0] and min(sizes) > sizes[0] / 3
    assert eps_n[-1] < 1.5 * eps_n[0]
