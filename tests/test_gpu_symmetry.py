"""Symmetries of the HIP path itself (no oracle): energies invariant and
forces / virials equivariant under rotations, reflections, translations
and permutations of the atoms, for the FP32 and BF16-MFMA paths; Newton's
third law (sum of forces zero) and zero net torque for clusters."""

import sys

import numpy as np
import pytest

import synth
from gpu_helpers import gpu_run, weights_for

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rotation(seed, reflect=False):
    rng = np.random.default_rng(seed)
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    if reflect:
        q = q @ np.diag([1.0, 1.0, -1.0])
    return q


def _transform(s, Q, t):
    """Positions r -> Q r + t; periodic cells rotate with them (rows a, b, c)."""
    import dataclasses
    pos = s.pos @ Q.T + t
    cell = np.einsum("bij,kj->bik", s.cell, Q)
    return dataclasses.replace(s, pos=pos, cell=cell)


# (config, structure): clusters (open) and a periodic lattice
CASES = {
    "C_clusters": lambda: ("C", synth.clusters(4, 30, 80, 0.1, 0.9, 10, 301)),
    "B_lattice": lambda: ("B", synth.cubic_lattice(5, 2.2, 0.25, 4, 302)),
}


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("name", list(CASES))
def test_rotation_translation_invariance(name, precision):
    cfg, s = CASES[name]()
    hp = synth.load_hparams(cfg)
    w = weights_for(hp, 41)
    a = gpu_run(hp, w, s, precision)
    # BF16: two evaluations round different inputs (~0.35 % force error each)
    tol = 2e-5 if precision == "fp32" else 1e-2
    for k, refl in ((0, False), (1, True)):
        Q = _rotation(500 + k, reflect=refl)
        b = gpu_run(hp, w, _transform(s, Q, np.array([0.37, -1.2, 2.5])), precision)
        de = np.abs(b["e_struct"] - a["e_struct"]).max() / s.n_atoms
        fr = np.linalg.norm(b["forces"] - a["forces"] @ Q.T) / np.linalg.norm(a["forces"])
        wr = np.linalg.norm(b["virial"] - np.einsum("ij,bjk,lk->bil", Q, a["virial"], Q)) / np.linalg.norm(a["virial"])
        _say(f"[sym] {name} {precision} reflect={refl}: |dE|/N {de:.2e} eV, F rel {fr:.2e}, W rel {wr:.2e}")
        assert de < (1e-5 if precision == "fp32" else 1e-3)
        assert fr < tol and wr < tol


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_permutation_invariance(precision):
    cfg, s = CASES["C_clusters"]()
    hp = synth.load_hparams(cfg)
    w = weights_for(hp, 42)
    a = gpu_run(hp, w, s, precision)
    # permute atoms within each structure (segments stay contiguous)
    import dataclasses
    rng = np.random.default_rng(77)
    perm = np.concatenate([s.seg[b] + rng.permutation(s.seg[b + 1] - s.seg[b]) for b in range(s.n_struct)])
    sp = dataclasses.replace(s, pos=s.pos[perm], species=s.species[perm])
    b = gpu_run(hp, w, sp, precision)
    tol = 1e-5 if precision == "fp32" else 1e-2
    assert np.abs(b["e_struct"] - a["e_struct"]).max() / s.n_atoms < (1e-5 if precision == "fp32" else 1e-3)
    fr = np.linalg.norm(b["forces"] - a["forces"][perm]) / np.linalg.norm(a["forces"])
    _say(f"[sym] permutation {precision}: F rel {fr:.2e}")
    assert fr < tol


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_newton_third_law_and_torque(precision):
    cfg, s = CASES["C_clusters"]()
    hp = synth.load_hparams(cfg)
    w = weights_for(hp, 43)
    a = gpu_run(hp, w, s, precision)
    F = a["forces"]
    scale = np.abs(F).max()
    for b in range(s.n_struct):
        sl = slice(s.seg[b], s.seg[b + 1])
        net = np.abs(F[sl].sum(0)).max()
        c = s.pos[sl] - s.pos[sl].mean(0)
        torque = np.abs(np.cross(c, F[sl]).sum(0)).max()
        # FP64 scatter of g_e - g_rev(e): exact cancellation up to FP64 rounding
        assert net < 1e-9 * scale * (s.seg[b + 1] - s.seg[b])
        assert torque < (1e-4 if precision == "fp32" else 3e-2) * scale * np.abs(c).max()
    _say(f"[sym] Newton/torque {precision} ok (max |F| {scale:.3f})")
