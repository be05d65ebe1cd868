"""l_max = 3 in full O(3) (the tensor features one degree above Table 1's
l = 2) through the C ABI: FP32 and BF16 energies, forces and virials
against the FP64 oracle for one- and two-layer models with 16 and 64
channels, non-unit path mixing and species scales, on a periodic lattice
spanning several edge tiles with a ragged tail and on a mixed batch of
triclinic cells and open clusters; the double backward refuses l_max = 3
before launching anything."""

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


MODELS = {
    # name: (n_layers, latent, channels, two-body widths)
    "L2_w64_c16": (2, 64, 16, [16, 32, 64]),
    "L1_w64_c16": (1, 64, 16, [16, 32, 64]),
    "L2_w256_c64": (2, 256, 64, [64, 128, 256]),
}
SYSTEMS = {
    "lattice_5cube": lambda: synth.cubic_lattice(5, 2.2, 0.25, 4, 161),
    "mixed_6": lambda: synth.mixed_batch(6, 8, 40, 0.1, 4, 162),
}


def _case(model, system):
    """Hyperparameters with n-bar from the lattice's edges per atom and the
    energy scale that makes the FP64 force RMS 1 eV/A (forces are linear in
    it), both measured with the oracle; reference results of the system."""
    key = (model, system)
    if key in _CACHE:
        return _CACHE[key]
    from oracle import model as M
    from oracle import neighbors as nb
    NL, w, c, tb = MODELS[model]
    hp = dict(n_species=4, l_max=3, n_layers=NL, latent=w, channels=c, n_bessel=8, poly_p=6,
              twobody=tb, latent_depth=3, edge_hidden=16, r_cut=4.5, avg_num_neighbors=1.0, energy_scale=1.0)
    lat = SYSTEMS["lattice_5cube"]()
    hp["avg_num_neighbors"] = float(nb.build(lat, hp["r_cut"])["j"].shape[0]) / lat.n_atoms
    w_ = weights_nonunit(hp, 163)
    s = SYSTEMS[system]()
    ref1 = M.energy_forces(M.HParams.from_dict(hp), w_, lat)
    hp["energy_scale"] = 1.0 / float(np.sqrt(np.mean(ref1["forces"] ** 2)))
    ref = M.energy_forces(M.HParams.from_dict(hp), w_, s)
    _CACHE[key] = (hp, s, w_, ref)
    return _CACHE[key]


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("system", list(SYSTEMS))
@pytest.mark.parametrize("model", list(MODELS))
def test_lmax3_matches_oracle(model, system, prec):
    hp, s, w, ref = _case(model, system)
    gpu = gpu_run(hp, w, s, prec)
    assert gpu["status"] == 0
    rep = parity_report(hp, w, s, gpu, ref)
    n_edges = int(gpu["calc"].nl.n_edges.item())
    _say(f"[lmax3 {model} {system} {prec}] {s.n_atoms} atoms, {n_edges} edges: "
         + ", ".join(f"{k} {v:.3g}" for k, v in rep.items()))
    if prec == "fp32":
        for k in ("e_atom", "forces", "virial"):
            assert rep[k] < 1e-5, (k, rep[k])
    else:
        assert rep["e_per_atom_abs"] <= 1e-3
        assert rep["force_rms_abs"] <= 0.02


def test_lmax3_second_order_is_refused():
    import torch
    import paper_2502_06073_amd as afm
    hp, s, w, _ = _case("L2_w64_c16", "lattice_5cube")
    calc = afm.Calculator(afm.Model(hp, w, precision="fp32"), afm.DeviceSystem.from_synth(s), second_order=True)
    calc.build_neighbors()
    calc.energy_forces()
    with pytest.raises(afm.AfmError, match="second-order tensor-product kernel not built"):
        calc.forces_backward(torch.ones(s.n_struct, dtype=torch.float64, device="cuda"), None)


def test_lmax3_tile_shapes_bitwise_equal():
    """The l_max = 3 chains of every edge-tile shape give the same bits."""
    import torch
    import paper_2502_06073_amd as afm
    hp, s, w, _ = _case("L2_w256_c64", "lattice_5cube")
    model = afm.Model(hp, w, precision="bf16")
    calc = afm.Calculator(model, afm.DeviceSystem.from_synth(s))
    calc.build_neighbors()
    res = []
    for shape in ((64, 8), (128, 16), (128, 8)):
        model.set_edge_tile(*shape)
        out = calc.energy_forces()
        torch.cuda.synchronize()
        res.append({k: v.cpu().numpy() for k, v in out.items()})
    for r in res[1:]:
        for k in ("e_atom", "e_struct", "forces", "virial"):
            np.testing.assert_array_equal(res[0][k], r[k], err_msg=k)
