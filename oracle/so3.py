"""Oracle real spherical harmonics and Clebsch-Gordan tensors (test
infrastructure only).

The paper's tensor features are e3nn irreps with l up to 2 in full O(3)
(Methodology / Model Training); it prints no convention, so this module fixes
one and derives everything else from it:

* Real spherical harmonics, component normalised (sum_m Y_lm^2 = 2l + 1), on a
  unit vector u = (x, y, z), m = -l..l:
    Y^0 = 1
    Y^1 = sqrt(3) (y, z, x)
    Y^2 = (sqrt15 xy, sqrt15 yz, sqrt5/2 (3z^2 - 1), sqrt15 xz, sqrt15/2 (x^2 - y^2))
    Y^3 = standard real (no Condon-Shortley phase) cubic harmonics, same
          normalisation, m = -3..3 (used only for l_max = 3 variants).
* D^l(R) is defined by Y^l(R u) = D^l(R) Y^l(u); obtained here by least squares
  over random unit vectors.
* C^{l1 l2 l3} is the real tensor invariant under D^{l1} x D^{l2} x D^{l3}
  (the null space of the stacked (D x D x D - I) for three random rotations),
  normalised to sum C^2 = 2 l3 + 1, with the sign fixed so that the first
  nonzero entry in row-major (m1, m2, m3) order is positive.

Pins (tests/test_oracle_so3.py): the closed forms, sum rules, parity,
C^{0ll} = I, C^{l0l} = I, C^{ll0} = I / sqrt(2l+1), C^{111} = cross / sqrt 2,
nonzero counts and the contraction constants of Y^{l1} (x) Y^{l2} -> Y^{l3}.
"""

from __future__ import annotations

import functools
import math

import numpy as np


def real_sh(l: int, u: np.ndarray) -> np.ndarray:
    """Y^l(u) for unit vectors u [..., 3] -> [..., 2l+1] (float64)."""
    x, y, z = u[..., 0], u[..., 1], u[..., 2]
    if l == 0:
        return np.ones(u.shape[:-1] + (1,))
    if l == 1:
        return math.sqrt(3.0) * np.stack([y, z, x], axis=-1)
    if l == 2:
        s15 = math.sqrt(15.0)
        return np.stack([s15 * x * y, s15 * y * z,
                         0.5 * math.sqrt(5.0) * (3.0 * z * z - 1.0),
                         s15 * x * z, 0.5 * s15 * (x * x - y * y)], axis=-1)
    if l == 3:
        # Real cubic harmonics (no Condon-Shortley phase), normalised to
        # sum_m Y^2 = 7 on the sphere.
        c3 = math.sqrt(35.0 / 8.0)
        c2 = math.sqrt(105.0)
        c1 = math.sqrt(21.0 / 8.0)
        c0 = math.sqrt(7.0) / 2.0
        return np.stack([
            c3 * y * (3.0 * x * x - y * y),
            c2 * x * y * z,
            c1 * y * (5.0 * z * z - 1.0),
            c0 * z * (5.0 * z * z - 3.0),
            c1 * x * (5.0 * z * z - 1.0),
            0.5 * c2 * z * (x * x - y * y),
            c3 * x * (x * x - 3.0 * y * y)], axis=-1)
    raise ValueError("l > 3 not supported")


def random_rotation(rng: np.random.Generator) -> np.ndarray:
    """Haar-random proper rotation from the QR of a Gaussian matrix."""
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))[None, :]
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def random_units(rng: np.random.Generator, n: int) -> np.ndarray:
    v = rng.standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def wigner_d(l: int, R: np.ndarray, n_pts: int = 64, seed: int = 7) -> np.ndarray:
    """D^l(R) with Y^l(R u) = D^l(R) Y^l(u), by least squares."""
    rng = np.random.Generator(np.random.PCG64(seed))
    u = random_units(rng, n_pts)
    A = real_sh(l, u)                 # [n, d]
    B = real_sh(l, u @ R.T)           # [n, d] = A @ D^T
    Dt, *_ = np.linalg.lstsq(A, B, rcond=None)
    return Dt.T


@functools.lru_cache(maxsize=None)
def cg(l1: int, l2: int, l3: int) -> np.ndarray:
    """Real CG tensor C[m1, m2, m3] (float64, read-only copy returned)."""
    if not (abs(l1 - l2) <= l3 <= l1 + l2):
        raise ValueError("triangle rule violated")
    rng = np.random.Generator(np.random.PCG64(11 + 100 * l1 + 10 * l2 + l3))
    d1, d2, d3 = 2 * l1 + 1, 2 * l2 + 1, 2 * l3 + 1
    rows = []
    for _ in range(3):
        R = random_rotation(rng)
        K = np.kron(np.kron(wigner_d(l1, R), wigner_d(l2, R)), wigner_d(l3, R))
        rows.append(K - np.eye(d1 * d2 * d3))
    M = np.concatenate(rows, axis=0)
    _, s, vt = np.linalg.svd(M)
    null = vt[-1]
    if s[-1] > 1e-9 or (len(s) > 1 and s[-2] < 1e-6):
        raise RuntimeError("invariant space is not one-dimensional")
    C = null.reshape(d1, d2, d3)
    C[np.abs(C) < 1e-12] = 0.0
    C = C * math.sqrt(d3 / float(np.sum(C * C)))
    flat = C.ravel()
    first = flat[np.nonzero(np.abs(flat) > 1e-9)[0][0]]
    if first < 0:
        C = -C
    C.setflags(write=False)
    return C
