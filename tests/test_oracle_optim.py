"""Pins of the oracle Adam update."""

import numpy as np

from oracle import optim


def test_first_step_closed_form():
    # after one step m_hat = g and v_hat = g^2, so the move is lr g / (|g| + eps)
    rng = np.random.default_rng(1)
    th = rng.standard_normal(50)
    g = rng.standard_normal(50)
    new, m1, m2 = optim.adam_step(th, g, np.zeros(50), np.zeros(50), 1, lr=0.01, eps=1e-3)
    np.testing.assert_allclose(th - new, 0.01 * g / (np.abs(g) + 1e-3), rtol=1e-12)
    np.testing.assert_allclose(m1, 0.1 * g, rtol=1e-15)
    np.testing.assert_allclose(m2, 0.001 * g * g, rtol=1e-12)


def test_moments_are_exponential_averages():
    rng = np.random.default_rng(2)
    gs = rng.standard_normal((6, 4))
    th, m1, m2 = np.zeros(4), np.zeros(4), np.zeros(4)
    for t, g in enumerate(gs, start=1):
        th, m1, m2 = optim.adam_step(th, g, m1, m2, t, lr=1e-3)
    w1 = np.array([0.1 * 0.9 ** (5 - k) for k in range(6)])
    w2 = np.array([0.001 * 0.999 ** (5 - k) for k in range(6)])
    np.testing.assert_allclose(m1, w1 @ gs, rtol=1e-12)
    np.testing.assert_allclose(m2, w2 @ (gs * gs), rtol=1e-12)


def test_minimises_a_quadratic():
    a = np.array([1.0, 4.0, 0.25])
    th, m1, m2 = np.array([3.0, -2.0, 5.0]), np.zeros(3), np.zeros(3)
    for t in range(1, 3001):
        th, m1, m2 = optim.adam_step(th, a * th, m1, m2, t, lr=0.01)
    assert np.abs(th).max() < 1e-3
