"""FP32 parity with the oracle over a grid of model shapes that the other
GPU tests do not all reach: l_max 0, 1 and 2, one to three layers, 8 and
32 channels, per-path and dense mixing, on a small mixed batch (a triclinic
cell and open clusters), energies, forces and virials to 1e-5."""

import sys

import numpy as np
import pytest

import synth
from gpu_helpers import gpu_run, parity_report, weights_nonunit

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


CASES = [(lm, nl, c, mix) for lm in (0, 1, 2) for nl in (1, 2, 3) for c in (8, 32)
         for mix in ("path", "dense") if not (mix == "dense" and nl == 1)]
_SYS = {}


def _system():
    if "s" not in _SYS:
        _SYS["s"] = synth.mixed_batch(3, 8, 24, 0.1, 3, 191)
    return _SYS["s"]


@pytest.mark.parametrize("lm,nl,c,mix", CASES)
def test_shape_grid_fp32(lm, nl, c, mix):
    from oracle import model as M
    s = _system()
    hp = dict(n_species=3, l_max=lm, n_layers=nl, latent=32, channels=c, n_bessel=8, poly_p=6,
              twobody=[16, 32], latent_depth=2, edge_hidden=16, r_cut=4.0, avg_num_neighbors=12.0,
              energy_scale=0.7, mixing=mix)
    w = weights_nonunit(hp, 192 + 7 * lm + 3 * nl + c)
    _say(f"[grid] l_max {lm}, {nl} layers, {c} channels, {mix}: {s.n_atoms} atoms")
    gpu = gpu_run(hp, w, s, "fp32")
    assert gpu["status"] == 0
    ref = M.energy_forces(M.HParams.from_dict(hp), w, s)
    rep = parity_report(hp, w, s, gpu, ref)
    _say(f"[grid] l_max {lm}, {nl} layers, {c} channels, {mix}: " + ", ".join(f"{k} {v:.2g}" for k, v in rep.items()))
    for k in ("e_atom", "forces", "virial"):
        assert rep[k] < 1e-5, (k, rep[k])
