"""The seeded input generators: the smooth analytic state and its exact gradients."""
import numpy as np

from paper_2402_02075_amd import meshgen as mg


def test_smooth_state_gradients_are_exact():
    x = np.random.default_rng(0).uniform(size=(40, 3))
    W, G = mg.smooth_state_and_gradients(x, seed=9, amp=0.07)
    np.testing.assert_array_equal(W, mg.random_smooth_state(x, seed=9, amp=0.07))
    h = 1e-5
    for d in range(3):
        e = np.zeros(3)
        e[d] = h
        fd = (mg.random_smooth_state(x + e, seed=9, amp=0.07) - mg.random_smooth_state(x - e, seed=9, amp=0.07)) / (2 * h)
        np.testing.assert_allclose(G[d::3], fd, rtol=0, atol=1e-8)
