"""A whole evaluation step (edge lists + energies + forces + virials of a
flattened batch of uneven structures) captured into a hipGraph and replayed:
every replay must equal the eager calls on the same positions bit for bit,
with eager work, synchronisations and in-place position updates between
the replays; and the replayed energies of the mixed batch against the FP64
oracle."""

import dataclasses
import sys

import numpy as np
import pytest

import synth
from gpu_helpers import weights_nonunit

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_eval_graph_replays_equal_eager(prec):
    import torch
    import paper_2502_06073_amd as afm
    from oracle import model as M
    hp = synth.load_hparams("D")
    s = synth.config_d(12)
    w = weights_nonunit(hp, 78)
    model = afm.Model(hp, w, precision=prec)
    sysd = afm.DeviceSystem.from_synth(s)
    cg = afm.Calculator(model, sysd)
    ce = afm.Calculator(model, sysd)      # eager twin: same positions, own list and workspace
    cg.build_neighbors()
    g = afm.EvalGraph(cg, rebuild=True, virial=True)
    rng = np.random.default_rng(5)
    for rep in range(4):
        if rep:
            # move the atoms in place (the graph reads them at replay time)
            d = torch.tensor(rng.uniform(-0.05, 0.05, size=(s.n_atoms, 3)), device="cuda")
            sysd.pos.add_(d)
            torch.cuda.synchronize()
            _ = float(sysd.pos.sum().item())
        out = g.replay()
        ce.build_neighbors()
        ref = ce.energy_forces()
        torch.cuda.synchronize()
        for k in ("e_atom", "e_struct", "forces", "virial"):
            np.testing.assert_array_equal(out[k].cpu().numpy(), ref[k].cpu().numpy(), err_msg=f"{k} rep {rep}")
        assert cg.status() == 0 and ce.status() == 0
        if rep == 3:
            s2 = dataclasses.replace(s, pos=sysd.pos.cpu().numpy())
            e_ref = M.energy_forces(M.HParams.from_dict(hp), w, s2, want_forces=False)["e_struct"]
            e = out["e_struct"].cpu().numpy()
            err = np.abs(e - e_ref) / np.diff(s.seg)
            _say(f"[graph {prec}] 4 replays bitwise equal to eager; |dE_s|/N vs FP64 max {err.max():.2e} eV/atom")
            assert err.max() < (1e-3 if prec == "bf16" else 1e-5)
