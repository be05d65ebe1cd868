"""Oracle Adam update (test infrastructure only).

The paper optimises the parameters with Adam (Model Training).  This is the
algorithm of Kingma and Ba (2015, Algorithm 1) with bias-corrected moments,
written out for a flat float64 parameter vector.

Pins (tests/test_oracle_optim.py): the first step moves every parameter by
lr * g / (|g| + eps') (closed form of the bias-corrected first step), the
moments follow their exponential-average definitions, and the iteration
minimises a convex quadratic.
"""

from __future__ import annotations

import numpy as np


def adam_step(theta: np.ndarray, grad: np.ndarray, m1: np.ndarray, m2: np.ndarray, t: int,
              lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """One Adam step at step count t >= 1; returns (theta, m1, m2) new arrays."""
    g = np.asarray(grad, dtype=np.float64)
    m1 = beta1 * m1 + (1.0 - beta1) * g
    m2 = beta2 * m2 + (1.0 - beta2) * g * g
    m_hat = m1 / (1.0 - beta1 ** t)
    v_hat = m2 / (1.0 - beta2 ** t)
    return theta - lr * m_hat / (np.sqrt(v_hat) + eps), m1, m2
