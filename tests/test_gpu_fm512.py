"""The 512-wide model of Table 1 (latent width 512, 128 tensor channels,
two-body MLP [128, 256, 512], l_max 2, 2 layers) through the C ABI: FP32
and BF16 energies, forces and virials against the FP64 oracle on a periodic
lattice spanning several edge tiles with a ragged tail, non-unit path
mixing and species scales, and the double backward (weight gradient and
dJ/dr).  (Tensor products run as two 64-channel groups;
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


D2_TOL = {"fp32": 1e-5, "bf16": 1.5e-2}   # relative norm of the weight gradient


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_fm512_second_order_matches_oracle(prec):
    """The double backward of the 512-wide model (its 128-channel tensor
    products as two 64-channel launches): the weight gradient of
    J = sum gE E + sum gF . F + sum gW : W against the FP64 oracle's double
    backward, and for the FP32 model also dJ/dr."""
    import torch
    import paper_2502_06073_amd as afm
    from oracle import model as M
    hp, s, w, _ = _case()
    rng = np.random.default_rng(9)
    gE = rng.standard_normal(s.n_struct)
    gF = rng.standard_normal((s.n_atoms, 3))
    gW = rng.standard_normal((s.n_struct, 3, 3))
    model = afm.Model(hp, w, precision=prec)
    calc = afm.Calculator(model, afm.DeviceSystem.from_synth(s), second_order=True)
    calc.build_neighbors()
    dev = "cuda"
    g, gp = calc.forces_backward(torch.tensor(gE, device=dev), torch.tensor(gF, device=dev),
                                 torch.tensor(gW, device=dev), want_pos=True)
    torch.cuda.synchronize()
    g = g.cpu().numpy().astype(np.float64)
    gp = gp.cpu().numpy()
    ref = M.vjp_weights(M.HParams.from_dict(hp), w, s, gE, gF, grad_virial=gW, want_pos=True)
    gr = ref["grad_weights"]
    err = np.linalg.norm(g - gr) / np.linalg.norm(gr)
    cos = float(g @ gr / (np.linalg.norm(g) * np.linalg.norm(gr)))
    errp = np.linalg.norm(gp - ref["grad_pos"]) / np.linalg.norm(ref["grad_pos"])
    lay = M.param_layout(M.HParams.from_dict(hp))
    worst, off = [], 0
    for b in lay:
        seg = slice(off, off + b["size"])
        den = max(np.linalg.norm(gr[seg]), 1e-30)
        worst.append((round(float(np.linalg.norm(g[seg] - gr[seg]) / den), 7), b["name"]))
        off += b["size"]
    worst.sort(reverse=True)
    _say(f"[fm512 d2 {prec}] weights rel {err:.2e}, cosine {cos:.7f}, grad_pos rel {errp:.2e}; "
         f"worst blocks {worst[:3]}")
    assert err < D2_TOL[prec] and cos > 0.999
    if prec == "fp32":
        assert worst[0][0] < 10 * D2_TOL[prec]
        assert errp < D2_TOL[prec]
    assert calc.status() == 0
