"""Edge-tile shapes of the BF16 MFMA chains (edges x wavefronts = 64 x 8,
128 x 16, 128 x 8): every output is bitwise the same with every shape (an
edge's MLP does not depend on the edges sharing its tile), also through the
split forward/backward calls and the fast adjoint, on inputs spanning
several tiles with ragged tails; all are within the BF16 gates
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


SHAPES = ((64, 8), (128, 16), (128, 8))


def _eval(calc, shape):
    import torch
    calc.model.set_edge_tile(*shape)
    assert calc.model.edge_tile == shape
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
    res = [_eval(calc, sh) for sh in SHAPES]
    for r in res[1:]:
        for k in ("e_atom", "e_struct", "forces", "virial"):
            np.testing.assert_array_equal(res[0][k], r[k], err_msg=k)
    # split forward / backward with weighted structures, every shape
    ges = torch.tensor(np.random.default_rng(3).uniform(0.5, 1.5, s.n_struct), device="cuda")
    split = []
    for sh in SHAPES:
        model.set_edge_tile(*sh)
        calc.forward_energy()
        F, W = calc.backward_forces(ges, virial=True)
        torch.cuda.synchronize()
        split.append((F.cpu().numpy(), W.cpu().numpy()))
    for x in split[1:]:
        np.testing.assert_array_equal(split[0][0], x[0])
        np.testing.assert_array_equal(split[0][1], x[1])
    ref = M.energy_forces(M.HParams.from_dict(hp), w, s)
    rep = parity_report(hp, w, s, res[2], ref)
    _say(f"[tiles {prec}] {name}: 64x8 == 128x16 == 128x8 bitwise; vs FP64 |dE_s|/N "
         f"{rep['e_per_atom_abs'] * 1e3:.3f} meV/atom, force RMS {rep['force_rms_abs'] * 1e3:.2f} meV/A")
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
    assert r1["tile"] in SHAPES and not r1["from_cache"]
    assert all(v > 0 for v in r1["ms"].values())
    best = min(SHAPES, key=lambda sh: r1["ms"][f"{sh[0]}x{sh[1]}"])
    assert r1["tile"] == best and model.edge_tile == best
    entries = json.loads(open(path).read())
    assert len(entries) == 1
    key = next(iter(entries))
    assert key.startswith("gfx950/w256/c64/l2/L2/d3/tb64-128-256/nb8/bf16/deg")
    assert (entries[key]["edges"], entries[key]["waves"]) == best
    # a second model of the same shape on the same workload: answered by the cache
    model2 = afm.Model(hp, w, precision="bf16")
    model2.set_edge_tile(*(SHAPES[0] if best != SHAPES[0] else SHAPES[1]))
    calc2 = afm.Calculator(model2, afm.DeviceSystem.from_synth(s))
    calc2.build_neighbors()
    r2 = calc2.tune_edge_tile(path)
    assert r2["from_cache"] and r2["tile"] == best and model2.edge_tile == best
    # FP32 models have no chains to tune
    m32 = afm.Model(hp, w, precision="fp32")
    c32 = afm.Calculator(m32, afm.DeviceSystem.from_synth(s))
    c32.build_neighbors()
    assert c32.tune_edge_tile(path)["tile"] == (0, 0) and m32.edge_tile == (0, 0)
