"""Pins of the oracle's spherical harmonics and Clebsch-Gordan tensors
against closed forms, scipy's complex spherical harmonics and sympy's exact
complex Clebsch-Gordan coefficients (all independent of the oracle code)."""

import math

import numpy as np
import pytest
import scipy.special as sps

from oracle import so3


def _units(n, seed=0):
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def _real_from_scipy(l, u):
    """Real, component-normalised SH without Condon-Shortley phase built from
    scipy's complex Y_l^m (which includes the phase)."""
    x, y, z = u[:, 0], u[:, 1], u[:, 2]
    theta = np.arccos(np.clip(z, -1, 1))
    phi = np.arctan2(y, x)
    out = []
    for m in range(-l, l + 1):
        Ylm = sps.sph_harm_y(l, abs(m), theta, phi)    # includes (-1)^m
        if m == 0:
            val = Ylm.real
        elif m > 0:
            val = math.sqrt(2) * (-1) ** m * Ylm.real
        else:
            val = math.sqrt(2) * (-1) ** m * Ylm.imag
        out.append(val * math.sqrt(4 * math.pi))
    return np.stack(out, axis=1)


@pytest.mark.parametrize("l", [0, 1, 2, 3])
def test_sh_matches_scipy(l):
    u = _units(200)
    np.testing.assert_allclose(so3.real_sh(l, u), _real_from_scipy(l, u),
                               atol=1e-12)


@pytest.mark.parametrize("l", [0, 1, 2, 3])
def test_sh_sum_rule_and_parity(l):
    u = _units(100, 1)
    Y = so3.real_sh(l, u)
    np.testing.assert_allclose((Y * Y).sum(1), 2 * l + 1, atol=1e-12)
    np.testing.assert_allclose(so3.real_sh(l, -u), (-1) ** l * Y, atol=1e-13)


def test_sh_l1_rotation_rule():
    rng = np.random.default_rng(3)
    R = so3.random_rotation(rng)
    P = np.array([[0, 1, 0], [0, 0, 1], [1, 0, 0]], float)   # (x,y,z)->(y,z,x)
    u = _units(50, 2)
    lhs = so3.real_sh(1, u @ R.T)
    rhs = so3.real_sh(1, u) @ (P @ R @ P.T).T
    np.testing.assert_allclose(lhs, rhs, atol=1e-13)


def test_sh_orthonormal_quadrature():
    # Gauss-Legendre in cos(theta) x uniform phi: exact for these degrees
    xg, wg = np.polynomial.legendre.leggauss(12)
    phis = np.arange(24) * 2 * math.pi / 24
    ct, ph = np.meshgrid(xg, phis, indexing="ij")
    wt = np.repeat(wg[:, None], 24, axis=1) * (2 * math.pi / 24) / (4 * math.pi)
    st = np.sqrt(1 - ct ** 2)
    u = np.stack([st * np.cos(ph), st * np.sin(ph), ct], -1).reshape(-1, 3)
    Y = np.concatenate([so3.real_sh(l, u) for l in range(4)], axis=1)
    G = (Y * wt.reshape(-1, 1)).T @ Y
    np.testing.assert_allclose(G, np.eye(16), atol=1e-12)


# ---------------------------------------------------------------- CG

TRIPLES = [(l1, l2, l3) for l1 in range(3) for l2 in range(3)
           for l3 in range(abs(l1 - l2), min(l1 + l2, 2) + 1)]

NNZ = {(0, 0, 0): 1, (0, 1, 1): 3, (0, 2, 2): 5, (1, 0, 1): 3, (1, 1, 0): 3,
       (1, 1, 1): 6, (1, 1, 2): 11, (1, 2, 1): 11, (1, 2, 2): 16,
       (2, 0, 2): 5, (2, 1, 1): 11, (2, 1, 2): 16, (2, 2, 0): 5,
       (2, 2, 1): 16, (2, 2, 2): 25}


def test_cg_nonzero_counts():
    assert sorted(NNZ) == sorted(TRIPLES)
    tot = 0
    for t in TRIPLES:
        n = int((np.abs(so3.cg(*t)) > 1e-12).sum())
        assert n == NNZ[t], t
        tot += n
    assert tot == 137


@pytest.mark.parametrize("l", [0, 1, 2])
def test_cg_closed_forms(l):
    d = 2 * l + 1
    np.testing.assert_allclose(so3.cg(0, l, l)[0], np.eye(d), atol=1e-12)
    np.testing.assert_allclose(so3.cg(l, 0, l)[:, 0, :], np.eye(d), atol=1e-12)
    np.testing.assert_allclose(so3.cg(l, l, 0)[:, :, 0], np.eye(d) / math.sqrt(d),
                               atol=1e-12)


def test_cg_111_is_cross_product():
    C = so3.cg(1, 1, 1)
    eps = np.zeros((3, 3, 3))
    for a, b, c in [(0, 1, 2), (1, 2, 0), (2, 0, 1)]:
        eps[a, b, c] = 1
        eps[a, c, b] = -1
    np.testing.assert_allclose(C, eps / math.sqrt(2), atol=1e-12)
    assert C[0, 1, 2] > 0


# contraction constants: sum C Y^l1(u) Y^l2(u) = k Y^l3(u)
K = {(0, 0, 0): 1.0, (0, 1, 1): 1.0, (1, 0, 1): 1.0, (0, 2, 2): 1.0,
     (2, 0, 2): 1.0, (1, 1, 0): math.sqrt(3), (1, 1, 2): -math.sqrt(6 / 5),
     (1, 2, 1): math.sqrt(2), (2, 1, 1): math.sqrt(2), (2, 2, 0): math.sqrt(5),
     (2, 2, 2): -math.sqrt(10 / 7)}


@pytest.mark.parametrize("t", TRIPLES)
def test_cg_contraction_constants(t):
    l1, l2, l3 = t
    u = _units(40, 5)
    C = so3.cg(*t)
    lhs = np.einsum("abk,ea,eb->ek", C, so3.real_sh(l1, u), so3.real_sh(l2, u))
    k = K.get(t, 0.0)
    if (l1 + l2 + l3) % 2:
        assert k == 0.0
    np.testing.assert_allclose(lhs, k * so3.real_sh(l3, u), atol=1e-12)


def _real_basis(l):
    """U with Y_real = U @ Y_complex (complex Y with Condon-Shortley phase)."""
    d = 2 * l + 1
    U = np.zeros((d, d), complex)
    for m in range(-l, l + 1):
        r = m + l
        if m == 0:
            U[r, l] = 1
        elif m > 0:
            U[r, l + m] = (-1) ** m / math.sqrt(2)
            U[r, l - m] = 1 / math.sqrt(2)
        else:
            U[r, l + abs(m)] = -1j * (-1) ** m / math.sqrt(2)
            U[r, l - abs(m)] = 1j / math.sqrt(2)
    return U


# every coupling the l_max = 3 models use (l <= 3)
TRIPLES3 = [(l1, l2, l3) for l1 in range(4) for l2 in range(4)
            for l3 in range(abs(l1 - l2), min(l1 + l2, 3) + 1)]


def test_cg_invariance_l3():
    """C^{l1 l2 l3} is invariant under D^{l1} x D^{l2} x D^{l3}, with D^l taken
    from the harmonics themselves (Y^l(R u) = D^l(R) Y^l(u), least squares over
    random directions), for every coupling with l <= 3."""
    rng = np.random.default_rng(11)
    R = so3.random_rotation(rng)
    u = _units(300, 12)
    D = {l: np.linalg.lstsq(so3.real_sh(l, u), so3.real_sh(l, u @ R.T), rcond=None)[0].T
         for l in range(4)}
    for t in TRIPLES3:
        l1, l2, l3 = t
        C = so3.cg(*t)
        rot = np.einsum("ia,jb,kc,abc->ijk", D[l1], D[l2], D[l3], C)
        np.testing.assert_allclose(rot, C, atol=1e-10, err_msg=str(t))
        np.testing.assert_allclose(np.sum(C ** 2), 2 * l3 + 1, atol=1e-12)


@pytest.mark.parametrize("t", TRIPLES3)
def test_cg_matches_sympy(t):
    """Real CG from sympy's exact complex coefficients, up to the convention
    (normalisation, sign of the first nonzero entry)."""
    sympy = pytest.importorskip("sympy")
    from sympy.physics.quantum.cg import CG
    l1, l2, l3 = t
    Cc = np.zeros((2 * l1 + 1, 2 * l2 + 1, 2 * l3 + 1))
    for m1 in range(-l1, l1 + 1):
        for m2 in range(-l2, l2 + 1):
            m3 = m1 + m2
            if abs(m3) <= l3:
                Cc[m1 + l1, m2 + l2, m3 + l3] = float(
                    CG(l1, m1, l2, m2, l3, m3).doit())
    # check the real-basis transform against scipy's SH first
    u = _units(30, 9)
    for l in (l1, l2, l3):
        x, y, z = u.T
        th, ph = np.arccos(z), np.arctan2(y, x)
        Yc = np.stack([sps.sph_harm_y(l, m, th, ph)
                       for m in range(-l, l + 1)], 1) * math.sqrt(4 * math.pi)
        np.testing.assert_allclose((Yc @ _real_basis(l).T).real,
                                   so3.real_sh(l, u), atol=1e-12)
    U1, U2, U3 = _real_basis(l1), _real_basis(l2), _real_basis(l3)
    # coupling: Y3(c) ~ sum CG Y1(c) Y2(c) -> real tensor
    Cr = np.einsum("ia,jb,kc,abc->ijk", U1.conj(), U2.conj(), U3, Cc)
    if np.abs(Cr.real).max() < 1e-12:
        Cr = Cr.imag
    else:
        assert np.abs(Cr.imag).max() < 1e-12
        Cr = Cr.real
    Cr = Cr * math.sqrt((2 * l3 + 1) / np.sum(Cr ** 2))
    flat = Cr.ravel()
    if flat[np.nonzero(np.abs(flat) > 1e-9)[0][0]] < 0:
        Cr = -Cr
    np.testing.assert_allclose(so3.cg(*t), Cr, atol=1e-12)
