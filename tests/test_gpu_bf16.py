"""GPU parity of the BF16-MFMA path against the FP64 oracle.

Tolerances (errors reported against FP64): total energy per atom
|E_s - E_s^ref| / N_s <= 1 meV and per-component force RMS <= 20 meV/A, on
workloads whose energy_scale is calibrated so the FP64 force RMS is
~1 eV/A.  The BF16 path must also be deterministic and chunk-invariant."""

import sys

import numpy as np
import pytest

import synth
from gpu_helpers import gpu_run, parity_report, weights_for

pytestmark = pytest.mark.gpu

E_TOL = 1e-3      # eV / atom
F_TOL = 0.020     # eV / A


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


CASES = {
    "A": lambda: ("A", synth.config_a()),
    "Bshape_5cube": lambda: ("B", synth.cubic_lattice(5, 2.2, 0.25, 4, 91)),
    "Bshape_8cube": lambda: ("B", synth.cubic_lattice(8, 2.2, 0.25, 4, 96)),
    "C_8clusters": lambda: ("C", synth.clusters(8, 20, 200, 0.1, 0.9, 10, 92)),
    "D_12mixed": lambda: ("D", synth.config_d(12)),
    "E_6cube": lambda: ("E", synth.cubic_lattice(6, 2.3, 0.25, 4, 97)),
}


@pytest.mark.parametrize("name,prec", [(n, "bf16") for n in CASES] +
                         [("Bshape_5cube", "bf16_fast"), ("D_12mixed", "bf16_fast"), ("E_6cube", "bf16_fast")])
def test_bf16_parity(name, prec):
    from oracle import model as M
    cfg, s = CASES[name]()
    hp = synth.load_hparams(cfg)
    w = synth.draw_weights(M.param_layout(M.HParams.from_dict(hp)), synth.WEIGHT_SEEDS[cfg])
    _say(f"[{prec}] {name} N={s.n_atoms}")
    r_list = hp.get("r_list", hp["r_cut"])
    gpu = gpu_run(hp, w, s, prec, r_list=r_list)
    assert gpu["status"] == 0
    ref = M.energy_forces(M.HParams.from_dict(hp), w, s, r_list=r_list)
    rep = parity_report(hp, w, s, gpu, ref)
    f_rms_ref = float(np.sqrt(np.mean(ref["forces"] ** 2)))
    _say(f"[{prec}] {name} {rep} ref-force-rms {f_rms_ref:.3f}")
    assert rep["e_per_atom_abs"] <= E_TOL, rep
    assert rep["force_rms_abs"] <= F_TOL, rep
    assert rep["forces"] <= 0.03, rep          # relative, scale-free


def test_bf16_matches_fp32_structure():
    """BF16 and FP32 paths agree to BF16 accuracy on the same inputs (both
    through the C ABI), so a layout bug in either would show."""
    cfg, s = CASES["Bshape_5cube"]()
    hp = synth.load_hparams(cfg)
    w = weights_for(hp, 17)
    a = gpu_run(hp, w, s, "bf16")
    b = gpu_run(hp, w, s, "fp32")
    rel = np.linalg.norm(a["forces"] - b["forces"]) / np.linalg.norm(b["forces"])
    _say(f"[bf16 vs fp32] force rel {rel:.3e}")
    assert rel < 0.03


def test_bf16_matches_fp32_dense_rows():
    """Rows of ~200 edges (three times the headline lattice's): the
    per-atom tensor-product kernels loop several times over their edge
    slots and the per-row reductions over several lane-group steps."""
    cfg = "B"
    hp = synth.load_hparams(cfg)
    s = synth.cubic_lattice(8, 1.5, 0.15, 4, 99)       # 12 A box, ~200 edges/row
    w = weights_for(hp, 19)
    a = gpu_run(hp, w, s, "bf16")
    b = gpu_run(hp, w, s, "fp32")
    assert a["status"] == 0 and b["status"] == 0
    rel = np.linalg.norm(a["forces"] - b["forces"]) / np.linalg.norm(b["forces"])
    _say(f"[bf16 vs fp32 dense] force rel {rel:.3e}")
    assert rel < 0.03


def test_bf16_deterministic_and_chunk_invariant():
    cfg = "B"
    hp = synth.load_hparams(cfg)
    s = synth.cubic_lattice(8, 2.2, 0.25, 4, 98)
    w = weights_for(hp, 18)
    a = gpu_run(hp, w, s, "bf16")
    b = gpu_run(hp, w, s, "bf16")
    c = gpu_run(hp, w, s, "bf16", max_bytes=300 * 2 ** 20)
    _say(f"[bf16 chunks] {c['n_chunks']}")
    assert c["n_chunks"] > 1
    for k in ("e_atom", "forces", "virial"):
        np.testing.assert_array_equal(a[k], b[k])
        np.testing.assert_array_equal(a[k], c[k])


def test_bf16_full_B_sampled_atoms():
    from oracle import model as M
    hp = synth.load_hparams("B")
    s = synth.config_b()
    w = synth.draw_weights(M.param_layout(M.HParams.from_dict(hp)), synth.WEIGHT_SEEDS["B"])
    gpu = gpu_run(hp, w, s, "bf16")
    assert gpu["status"] == 0
    atoms = synth.subset_rows(s.n_atoms, 12, 101)
    ref = M.forces_subset(M.HParams.from_dict(hp), w, s, atoms)
    d = gpu["forces"][atoms] - ref["forces"]
    rms = float(np.sqrt(np.mean(d * d)))
    de = np.abs(gpu["e_atom"][atoms] - ref["e_atom"])
    _say(f"[bf16 B sample] force rms err {rms:.4f} eV/A, per-atom |dE| max {de.max():.4f} eV")
    assert rms <= F_TOL
