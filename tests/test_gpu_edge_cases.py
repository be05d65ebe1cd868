"""Degenerate inputs through the C ABI: isolated atoms and structures
without edges (their energy is the species shift, their force zero), an
edge list that overflows its capacity (flag set, required count reported,
energies NaN, nothing read past a buffer), and species indices out of range
(flag set, only the affected atom's energy is NaN)."""

import sys

import numpy as np
import pytest

import synth
from gpu_helpers import gpu_run, mu_of, weights_for

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _degenerate_batch(hp):
    S = hp["n_species"]
    rc = hp["r_cut"]
    open3 = (np.zeros((1, 3, 3)), np.zeros(1, np.uint8))
    lone = synth.System(np.zeros((1, 3)), np.array([1 % S], np.int32), *open3, np.array([0, 1], np.int64), S)
    far = synth.System(np.array([[0.0, 0, 0], [rc + 0.5, 0.3, -0.2]]), np.array([0, 2 % S], np.int32), *open3,
                       np.array([0, 2], np.int64), S)
    dimer = synth.System(np.array([[0.0, 0, 0], [1.1, 1.2, 0.4]]), np.array([0, 1 % S], np.int32), *open3,
                         np.array([0, 2], np.int64), S)
    cl = synth.clusters(1, 12, 12, 0.1, 0.9, S, 121)
    return synth._pack([lone, far, dimer, cl, lone], S)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_isolated_atoms_and_structures_without_edges(prec):
    from oracle import model as M
    hp = synth.load_hparams("C")
    s = _degenerate_batch(hp)
    w = weights_for(hp, 51)
    gpu = gpu_run(hp, w, s, prec)
    assert gpu["status"] == 0
    ref = M.energy_forces(M.HParams.from_dict(hp), w, s)
    mu = mu_of(hp, w, s)
    iso = [0, 1, 2, s.n_atoms - 1]                   # the lone atoms and the far dimer
    np.testing.assert_allclose(gpu["e_atom"][iso], mu[iso], rtol=1e-12, atol=1e-12)
    np.testing.assert_array_equal(gpu["forces"][iso], 0.0)
    np.testing.assert_array_equal(gpu["virial"][[0, 1, 4]], 0.0)
    tol = 1e-5 if prec == "fp32" else 3e-2
    ea = np.linalg.norm((gpu["e_atom"] - mu) - (ref["e_atom"] - mu)) / np.linalg.norm(ref["e_atom"] - mu)
    fr = np.linalg.norm(gpu["forces"] - ref["forces"]) / np.linalg.norm(ref["forces"])
    _say(f"[edge {prec}] isolated atoms exact; e_atom rel {ea:.2e}, forces rel {fr:.2e}")
    assert ea < tol and fr < tol


def test_capacity_overflow_is_flagged():
    import torch
    import paper_2502_06073_amd as afm
    hp = synth.load_hparams("C")
    s = synth.clusters(4, 20, 60, 0.1, 0.9, 10, 122)
    w = weights_for(hp, 52)
    full = gpu_run(hp, w, s, "fp32")
    need = int(full["calc"].nl.n_edges.item())
    small = afm.Calculator(afm.Model(hp, w, precision="fp32"), afm.DeviceSystem.from_synth(s),
                           r_list=hp["r_cut"], capacity=need // 2)
    small.build_neighbors()
    out = small.energy_forces()
    torch.cuda.synchronize()
    st = small.status()
    _say(f"[edge capacity] need {need}, capacity {need // 2}: status {st}, n_edges {int(small.nl.n_edges.item())}")
    assert st & 1
    assert int(small.nl.n_edges.item()) == need
    assert np.isnan(out["e_atom"].cpu().numpy()).all()
    assert np.isnan(out["forces"].cpu().numpy()).all()


def test_species_out_of_range_is_flagged():
    import torch
    import paper_2502_06073_amd as afm
    hp = synth.load_hparams("C")
    s = synth.clusters(2, 20, 30, 0.1, 0.9, 10, 123)
    bad = s.species.copy()
    bad[5] = hp["n_species"]          # one past the last species
    s2 = synth.System(s.pos, bad, s.cell, s.pbc, s.seg, s.n_species)
    w = weights_for(hp, 53)
    calc = afm.Calculator(afm.Model(hp, w, precision="fp32"), afm.DeviceSystem.from_synth(s2),
                          r_list=hp["r_cut"])
    calc.build_neighbors()
    out = calc.energy_forces()
    torch.cuda.synchronize()
    ea = out["e_atom"].cpu().numpy()
    _say(f"[edge species] status {calc.status()}; NaN energies at {np.flatnonzero(np.isnan(ea)).tolist()}")
    assert calc.status() & 4
    assert np.isnan(ea[5]) and np.isfinite(np.delete(ea, 5)).all()
