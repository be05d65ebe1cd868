"""The 512-wide model of Table 1 (latent width 512, 128 tensor channels,
two-body MLP [128, 256, 512], l_max 2, 2 layers) through the C ABI: FP32
and BF16 energies, forces and virials against the FP64 oracle on a periodic
lattice spanning several edge tiles with a ragged tail, non-unit path
mixing and species scales.  (Tensor products run as two 64-channel groups;
the MLP chains give each wavefront two output-row pairs.)"""

import sys

import numpy as np
import pytest

import synth
from gpu_helpers import gpu_run, parity_report, weights_nonunit

pytestmark = pytest.mark.gpu
_CACHE = {}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _case():
    """FM512 hyperparameters; n-bar from the lattice's edges per atom and the
    energy scale that makes the FP64 force RMS 1 eV/A (forces are linear in
    it), both measured with the oracle."""
    if "case" in _CACHE:
        return _CACHE["case"]
    from oracle import model as M
    from oracle import neighbors as nb
    s = synth.cubic_lattice(5, 2.2, 0.25, 4, 151)
    hp = dict(n_species=4, l_max=2, n_layers=2, latent=512, channels=128, n_bessel=8, poly_p=6,
              twobody=[128, 256, 512], latent_depth=3, edge_hidden=128, r_cut=5.2,
              avg_num_neighbors=1.0, energy_scale=1.0)
    hp["avg_num_neighbors"] = float(nb.build(s, hp["r_cut"])["j"].shape[0]) / s.n_atoms
    w = weights_nonunit(hp, 152)
    ref1 = M.energy_forces(M.HParams.from_dict(hp), w, s)
    hp["energy_scale"] = 1.0 / float(np.sqrt(np.mean(ref1["forces"] ** 2)))
    ref = M.energy_forces(M.HParams.from_dict(hp), w, s)
    _CACHE["case"] = (hp, s, w, ref)
    return _CACHE["case"]


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_fm512_matches_oracle(prec):
    hp, s, w, ref = _case()
    gpu = gpu_run(hp, w, s, prec)
    assert gpu["status"] == 0
    rep = parity_report(hp, w, s, gpu, ref)
    n_edges = int(gpu["calc"].nl.n_edges.item())
    _say(f"[fm512 {prec}] {s.n_atoms} atoms, {n_edges} edges: {rep}")
    if prec == "fp32":
        for k in ("e_atom", "forces", "virial"):
            assert rep[k] < 1e-5, (k, rep[k])
    else:
        assert rep["e_per_atom_abs"] <= 1e-3
        assert rep["force_rms_abs"] <= 0.02
    assert gpu["calc"].model.edge_tile == ((64, 8) if prec == "bf16" else (0, 0))


def test_fm512_tiles_and_tuner():
    import paper_2502_06073_amd as afm
    hp, s, w, _ = _case()
    model = afm.Model(hp, w, precision="bf16")
    with pytest.raises(afm.AfmError):
        model.set_edge_tile(128, 16)
    calc = afm.Calculator(model, afm.DeviceSystem.from_synth(s))
    calc.build_neighbors()
    r = calc.tune_edge_tile()
    _say(f"[fm512 tuner] {r}")
    assert r["tile"] == (64, 8) and r["ms"]["128x16"] == -1.0 and r["ms"]["128x8"] == -1.0


def test_fm512_second_order_is_refused():
    """The double backward has no 128-channel tensor-product kernels: the
    call fails with an error instead of running anything else."""
    import torch
    import paper_2502_06073_amd as afm
    hp, s, w, _ = _case()
    model = afm.Model(hp, w, precision="fp32")
    calc = afm.Calculator(model, afm.DeviceSystem.from_synth(s), second_order=True)
    calc.build_neighbors()
    calc.energy_forces()
    gE = torch.ones(s.n_struct, dtype=torch.float64, device="cuda")
    with pytest.raises(afm.AfmError, match="second-order tensor-product kernel not built"):
        calc.forces_backward(gE, None)
