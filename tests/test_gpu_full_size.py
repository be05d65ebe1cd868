"""Full-size parity on the seeded workloads as the benchmark runs them:

* the whole edge lists of the 13,824-atom lattice, the 64 clusters and the
  512 uneven structures, bit for bit against the oracle's lists;
* the energies of every structure (and of 512 sampled atoms of the lattice)
  against FP64 oracle values stored in tests/golden/full_size_energies.json
  (written by tests/golden/make_full_size.py, oracle only): FP32 within
  1e-5 relative, BF16 within 1 meV/atom of |dE_s| / N_s.
"""

import json
import os
import sys

import numpy as np
import pytest

import synth
from gpu_helpers import gpu_nlist, gpu_run

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = json.load(open(os.path.join(HERE, "golden", "full_size_energies.json")))


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _weights(name):
    from oracle import model as M
    hp = synth.load_hparams(name)
    return hp, synth.draw_weights(M.param_layout(M.HParams.from_dict(hp)), synth.WEIGHT_SEEDS[name])


@pytest.mark.parametrize("name", ["B", "C", "D"])
def test_full_size_neighbor_lists_bit_exact(name):
    from oracle import neighbors as nb
    hp, w = _weights(name)
    s = synth.SYSTEMS[name]()
    _say(f"[full nl] {name}: {s.n_atoms} atoms, {s.n_struct} structures")
    gpu = gpu_run(hp, w, s, "fp32")
    assert gpu["status"] == 0
    g = gpu_nlist(gpu["calc"])
    ref = nb.build(s, hp.get("r_list", hp["r_cut"]))
    assert g["j"].shape[0] == GOLD[name]["n_edges"] == ref["j"].shape[0]
    np.testing.assert_array_equal(g["row_ptr"], ref["row_ptr"])
    np.testing.assert_array_equal(g["j"], ref["j"])
    np.testing.assert_array_equal(g["n"], ref["n"])
    np.testing.assert_array_equal(g["rev"], ref["rev"])


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("name", ["B", "C", "D"])
def test_full_size_energies(name, prec):
    hp, w = _weights(name)
    s = synth.SYSTEMS[name]()
    gpu = gpu_run(hp, w, s, prec)
    assert gpu["status"] == 0
    gold = GOLD[name]
    e_ref = np.asarray(gold["e_struct"])
    e = gpu["e_struct"]
    n_s = np.diff(s.seg).astype(np.float64)
    per_atom = np.abs(e - e_ref) / n_s
    mean_err = float(np.sum(e - e_ref) / np.sum(n_s))
    rel = float(np.linalg.norm(e - e_ref) / np.linalg.norm(e_ref))
    msg = (f"[full E {prec}] {name}: {s.n_struct} structures, max |dE_s|/N_s {per_atom.max() * 1e3:.4f} meV/atom, "
           f"batch mean {mean_err * 1e3:.4f} meV/atom, rel {rel:.2e}")
    if "e_atom" in gold:
        rows = np.asarray(gold["e_atom_rows"])
        de = gpu["e_atom"][rows] - np.asarray(gold["e_atom"])
        msg += f"; sampled E_i max |dE_i| {np.abs(de).max() * 1e3:.4f} meV, mean {de.mean() * 1e3:.4f} meV"
    _say(msg)
    if prec == "fp32":
        assert rel < 1e-5
        if "e_atom" in gold:
            assert np.linalg.norm(de) / np.linalg.norm(np.asarray(gold["e_atom"])) < 1e-5
    else:
        assert per_atom.max() <= 1e-3
