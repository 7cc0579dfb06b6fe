"""Host logic of the moment-driven lens rule: the general quadratic against
the drift-gap closed form in Twiss parameters, and the waist it promises
checked by transporting the covariance with the matrices."""
import math

import numpy as np
import pytest

from paper_2402_17248_amd.optimize import twiss_from_moments, waist_lens_strength


def cov21_of(beta, alpha, eps):
    c = [0.0] * 21
    c[0], c[3], c[15] = beta * eps, -alpha * eps, (1 + alpha * alpha) / beta * eps
    return c


def drift(d):
    return ((1.0, d), (0.0, 1.0))


def exit_x_cov(cov21, m1, q, m2):
    s = np.array([[cov21[0], cov21[3]], [cov21[3], cov21[15]]])
    m = np.array(m2) @ np.array([[1.0, 0.0], [-q, 1.0]]) @ np.array(m1)
    return m @ s @ m.T


@pytest.mark.parametrize("beta,alpha,d1,d2", [(3.2e-3, 0.0, 6.65, 6.65), (3.2e-3, 0.4, 5.0, 8.3),
                                             (1.0, -1.5, 2.0, 3.0)])
def test_drift_gap_matches_twiss_closed_form(beta, alpha, d1, d2):
    c = cov21_of(beta, alpha, 2e-9)
    q = waist_lens_strength(c, drift(d1), drift(d2))
    gam = (1 + alpha * alpha) / beta
    bl, al = beta - 2 * alpha * d1 + gam * d1 * d1, alpha - gam * d1
    a = (bl + math.sqrt(bl * bl - 4 * d2 * d2)) / (2 * d2)
    assert q == pytest.approx((a - al) / bl, rel=1e-9)
    s = exit_x_cov(c, drift(d1), q, drift(d2))
    assert abs(s[0, 1]) / math.sqrt(np.linalg.det(s)) < 1e-6          # alpha = 0 at the entrance


def test_general_sections_reach_a_waist_and_pick_the_small_one():
    rng = np.random.default_rng(3)
    for _ in range(20):
        a, b, c_ = rng.uniform(0.5, 2.0), rng.uniform(1.0, 8.0), rng.normal(scale=0.2)
        m1 = np.array([[a, b], [c_, (1 + b * c_) / a]])          # det 1
        m2 = np.array([[1.0, 4.0], [-0.05, 0.8]])
        m2[1] /= np.linalg.det(m2)
        c = cov21_of(2e-3, 0.3, 1e-9)
        try:
            q = waist_lens_strength(c, m1.tolist(), m2.tolist())
        except ValueError:
            continue
        s = exit_x_cov(c, m1, q, m2)
        eps = math.sqrt(np.linalg.det(s))
        assert abs(s[0, 1]) / eps < 1e-6
        # the other waist (if any) is not smaller
        for dq in np.linspace(-2, 2, 81):
            t = exit_x_cov(c, m1, q + dq, m2)
            if abs(t[0, 1]) / eps < 1e-3:
                assert t[0, 0] >= s[0, 0] * (1 - 1e-6)


def test_twiss_from_moments_round_trip():
    b, a, e = twiss_from_moments(cov21_of(0.7, -2.0, 3e-8))
    assert (b, a, e) == pytest.approx((0.7, -2.0, 3e-8), rel=1e-12)


def test_train_concurrently_rejects_a_shared_network():
    """Two jobs on one network handle would race on its buffers: rejected
    before anything runs (no GPU needed)."""
    import pytest
    from paper_2402_17248_amd.chain import train_concurrently

    class Net:
        def train(self, *a, **k):
            raise AssertionError("must not run")

    net = Net()
    with pytest.raises(ValueError, match="more than one job"):
        train_concurrently([(net, None, None, 0, {}), (net, None, None, 0, {})])
    assert train_concurrently([]) == []
