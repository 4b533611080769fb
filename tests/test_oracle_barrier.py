"""Pins for the oracle's IPC barrier (Sec. 3, equation barrier)."""
import numpy as np

from oracle import barrier

DHAT = 1e-3


def test_closed_form_value():
    # log(d/dhat) = -1 at d = dhat/e, so b = (dhat - dhat/e)^2
    d = DHAT / np.e
    assert np.isclose(barrier.b(np.array([d]), DHAT)[0], (DHAT - d) ** 2, rtol=1e-14)


def test_zero_outside_and_c2_at_dhat():
    d = np.array([DHAT, 2 * DHAT, 10.0])
    assert np.all(barrier.b(d, DHAT) == 0) and np.all(barrier.db(d, DHAT) == 0) \
        and np.all(barrier.d2b(d, DHAT) == 0)
    # approaching dhat from below all three go to zero (C^2 continuity)
    eps = 1e-7
    d = np.array([DHAT * (1 - eps)])
    assert abs(barrier.b(d, DHAT)[0]) < 1e-25
    assert abs(barrier.db(d, DHAT)[0]) < 1e-16
    assert abs(barrier.d2b(d, DHAT)[0]) < 1e-5


def test_derivatives_match_finite_differences():
    d = np.linspace(0.02, 0.98, 49) * DHAT
    e = 1e-7 * DHAT
    fd1 = (barrier.b(d + e, DHAT) - barrier.b(d - e, DHAT)) / (2 * e)
    fd2 = (barrier.db(d + e, DHAT) - barrier.db(d - e, DHAT)) / (2 * e)
    np.testing.assert_allclose(barrier.db(d, DHAT), fd1, rtol=1e-6, atol=1e-12)
    np.testing.assert_allclose(barrier.d2b(d, DHAT), fd2, rtol=1e-6)


def test_signs_on_active_range():
    d = np.linspace(1e-4, 1 - 1e-4, 1000) * DHAT
    assert np.all(barrier.b(d, DHAT) > 0)
    assert np.all(barrier.db(d, DHAT) < 0)        # repulsive
    assert np.all(barrier.d2b(d, DHAT) > 0)       # convex in d
    # the tangential term b'/d dominates b'' near contact (why eq9 is indefinite)
    dd = np.array([0.1 * DHAT])
    assert barrier.db(dd, DHAT)[0] / dd[0] < -barrier.d2b(dd, DHAT)[0] * 0.9
