"""Edge-tile shapes of the BF16 MFMA chains (64 edges x 8 wavefronts and
128 edges x 16 wavefronts): every output is bitwise the same with either
shape (an edge's MLP does not depend on the edges sharing its tile), also
through the split forward/backward calls and the fast adjoint, on inputs
spanning several tiles with ragged tails; both are within the BF16 gates
against the FP64 oracle; and the tuner picks a shape, writes its cache and
answers the next call from it."""

import json
import sys

import numpy as np
import pytest

import synth
from gpu_helpers import parity_report, weights_nonunit

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


CASES = {
    "Bshape_7cube": lambda: (synth.load_hparams("B"), synth.cubic_lattice(7, 2.2, 0.25, 4, 141)),
    "D_12mixed": lambda: (synth.load_hparams("D"), synth.config_d(12)),
}


def _eval(calc, tile):
    import torch
    calc.model.set_edge_tile(tile)
    assert calc.model.edge_tile == tile
    out = calc.energy_forces()
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


@pytest.mark.parametrize("prec", ["bf16", "bf16_fast"])
@pytest.mark.parametrize("name", list(CASES))
def test_tile_shapes_bitwise_equal(name, prec):
    import torch
    import paper_2502_06073_amd as afm
    from oracle import model as M
    hp, s = CASES[name]()
    w = weights_nonunit(hp, 142)
    model = afm.Model(hp, w, precision=prec)
    calc = afm.Calculator(model, afm.DeviceSystem.from_synth(s))
    calc.build_neighbors()
    a = _eval(calc, 64)
    b = _eval(calc, 128)
    for k in ("e_atom", "e_struct", "forces", "virial"):
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)
    # split forward / backward with weighted structures, 128-edge tiles
    ges = torch.tensor(np.random.default_rng(3).uniform(0.5, 1.5, s.n_struct), device="cuda")
    model.set_edge_tile(128)
    calc.forward_energy()
    f128 = calc.backward_forces(ges, virial=True)
    model.set_edge_tile(64)
    calc.forward_energy()
    f64 = calc.backward_forces(ges, virial=True)
    torch.cuda.synchronize()
    for x, y in zip(f64, f128):
        np.testing.assert_array_equal(x.cpu().numpy(), y.cpu().numpy())
    ref = M.energy_forces(M.HParams.from_dict(hp), w, s)
    rep = parity_report(hp, w, s, b, ref)
    _say(f"[tiles {prec}] {name}: 64 == 128 bitwise; vs FP64 |dE_s|/N {rep['e_per_atom_abs'] * 1e3:.3f} meV/atom, "
         f"force RMS {rep['force_rms_abs'] * 1e3:.2f} meV/A")
    assert rep["e_per_atom_abs"] <= 1e-3 and rep["force_rms_abs"] <= 0.02
    assert calc.status() == 0


def test_tuner_picks_a_shape_and_caches_it(tmp_path):
    import paper_2502_06073_amd as afm
    hp, s = CASES["Bshape_7cube"]()
    w = weights_nonunit(hp, 143)
    model = afm.Model(hp, w, precision="bf16")
    calc = afm.Calculator(model, afm.DeviceSystem.from_synth(s))
    calc.build_neighbors()
    path = str(tmp_path / "tiles.json")
    r1 = calc.tune_edge_tile(path)
    _say(f"[tuner] {r1}")
    assert r1["tile"] in (64, 128) and not r1["from_cache"]
    assert r1["ms_64"] > 0 and r1["ms_128"] > 0
    assert r1["tile"] == (128 if r1["ms_128"] < r1["ms_64"] else 64)
    assert model.edge_tile == r1["tile"]
    text = open(path).read()
    entries = json.loads(text)
    assert len(entries) == 1
    key = next(iter(entries))
    assert key.startswith("gfx950/w256/c64/l2/L2/d3/tb64-128-256/nb8/bf16/deg")
    assert entries[key]["tile"] == r1["tile"]
    # a second model of the same shape on the same workload: answered by the cache
    model2 = afm.Model(hp, w, precision="bf16")
    model2.set_edge_tile(128 if r1["tile"] == 64 else 64)
    calc2 = afm.Calculator(model2, afm.DeviceSystem.from_synth(s))
    calc2.build_neighbors()
    r2 = calc2.tune_edge_tile(path)
    assert r2["from_cache"] and r2["tile"] == r1["tile"] and model2.edge_tile == r1["tile"]
    # FP32 models have no chains to tune
    m32 = afm.Model(hp, w, precision="fp32")
    c32 = afm.Calculator(m32, afm.DeviceSystem.from_synth(s))
    c32.build_neighbors()
    assert c32.tune_edge_tile(path)["tile"] == 0 and m32.edge_tile == 0
