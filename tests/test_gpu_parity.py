"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Integer outputs (the edge list) must match bit for bit.  FP32 results must
be within 1e-5 relative (norm-wise, on the non-constant part of the
energies, forces and virials).  Sizes span several tiles and ragged tails;
the full 13,824-atom workload is checked on a seeded sample of atoms."""

import dataclasses
import sys

import numpy as np
import pytest

import synth
from gpu_helpers import gpu_nlist, gpu_run, parity_report, weights_for

pytestmark = pytest.mark.gpu

FP32_TOL = 1e-5


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _oracle_nl(s, r):
    from oracle import neighbors as nb
    return nb.build(s, r)


def _check_nl(gpu, ref):
    np.testing.assert_array_equal(gpu["row_ptr"], ref["row_ptr"])
    np.testing.assert_array_equal(gpu["j"], ref["j"])
    np.testing.assert_array_equal(gpu["n"], ref["n"])
    np.testing.assert_array_equal(gpu["rev"], ref["rev"])


def small_l2(**kw):
    d = dict(n_species=4, l_max=2, n_layers=2, latent=64, channels=16, n_bessel=8, poly_p=6,
             twobody=[16, 32, 64], latent_depth=3, edge_hidden=32, r_cut=5.5,
             avg_num_neighbors=72.5, energy_scale=3.0)
    d.update(kw)
    return d


CASES = {
    "A": lambda: (synth.load_hparams("A"), synth.config_a()),
    "Bshape_5cube": lambda: (synth.load_hparams("B"), synth.cubic_lattice(5, 2.2, 0.25, 4, 91)),
    "C_8clusters": lambda: (synth.load_hparams("C"), synth.clusters(8, 20, 200, 0.1, 0.9, 10, 92)),
    "D_12mixed": lambda: (synth.load_hparams("D"), synth.config_d(12)),
    "l2_c16_lattice": lambda: (small_l2(), synth.cubic_lattice(7, 2.2, 0.25, 4, 93)),
    # one structure of 1,331 atoms: more atoms than threads in a structure-sum
    # block, so its energy and virial sums take two strided terms per thread
    "l2_c16_11cube": lambda: (small_l2(), synth.cubic_lattice(11, 2.2, 0.25, 4, 102)),
}


@pytest.mark.parametrize("name", list(CASES))
def test_neighbors_bit_exact(name):
    hp, s = CASES[name]()
    _say(f"[nl] {name} N={s.n_atoms} B={s.n_struct}")
    gpu = gpu_run(hp, weights_for(hp, 5), s, "fp32")
    assert gpu["status"] == 0
    _check_nl(gpu_nlist(gpu["calc"]), _oracle_nl(s, hp["r_list"] if "r_list" in hp else hp["r_cut"]))


@pytest.mark.parametrize("kind", ["cubic_12", "triclinic_binned"])
def test_neighbors_bit_exact_binned(kind):
    """Structures large enough for the binned candidate search (at least
    3 bins per cell direction and 64 atoms): the list must still equal the
    oracle's bit for bit, canonical order and reverse index included."""
    import torch
    import paper_2502_06073_amd as afm
    if kind == "cubic_12":
        s, r = synth.cubic_lattice(12, 2.2, 0.25, 4, 95), 5.5
    else:
        d = synth.config_d(40)
        big = max((b for b in range(d.n_struct) if d.pbc[b]), key=lambda b: d.seg[b + 1] - d.seg[b])
        s, r = d.structure(big), 4.0
    # the binned search needs >= 3 bins of width >= r along every cell direction
    h = s.cell[0]
    vol = abs(np.linalg.det(h))
    widths = [vol / np.linalg.norm(np.cross(h[(k + 1) % 3], h[(k + 2) % 3])) for k in range(3)]
    assert min(widths) >= 3 * r and s.n_atoms >= 64, (widths, s.n_atoms)
    sysd = afm.DeviceSystem.from_synth(s)
    hp = small_l2(r_cut=r)
    model = afm.Model(hp, weights_for(hp, 8), precision="fp32")
    calc = afm.Calculator(model, sysd, r_list=r)
    calc.build_neighbors()
    torch.cuda.synchronize()
    _say(f"[nl binned] {kind} N={s.n_atoms} edges {int(calc.nl.n_edges.item())}")
    assert calc.status() == 0
    _check_nl(gpu_nlist(calc), _oracle_nl(s, r))


def test_neighbors_unwrapped_and_skin():
    s = synth.cubic_lattice(7, 2.3, 0.25, 4, 94)
    rng = np.random.default_rng(0)
    k = rng.integers(-2, 3, size=(s.n_atoms, 3))
    from oracle import neighbors as nb
    s = dataclasses.replace(s, pos=s.pos + nb.shift_vectors(s.cell[0], k))
    hp = small_l2(r_cut=5.5)
    gpu = gpu_run(hp, weights_for(hp, 6), s, "fp32", r_list=6.0)
    assert gpu["status"] == 0
    _check_nl(gpu_nlist(gpu["calc"]), nb.build(s, 6.0))


@pytest.mark.parametrize("name", list(CASES))
def test_fp32_parity(name):
    from oracle import model as M
    hp, s = CASES[name]()
    w = weights_for(hp, 7)
    _say(f"[fp32] {name} N={s.n_atoms}")
    gpu = gpu_run(hp, w, s, "fp32")
    ref = M.energy_forces(M.HParams.from_dict(hp), w, s)
    rep = parity_report(hp, w, s, gpu, ref)
    _say(f"[fp32] {name} {rep}")
    for k in ("e_atom", "e_struct", "forces", "virial"):
        assert rep[k] <= FP32_TOL, (k, rep)


def test_fp32_chunked_equals_single_chunk():
    hp = synth.load_hparams("B")
    s = synth.cubic_lattice(8, 2.2, 0.25, 4, 95)         # ~37k edges
    w = weights_for(hp, 8)
    one = gpu_run(hp, w, s, "fp32")
    many = gpu_run(hp, w, s, "fp32", max_bytes=400 * 2 ** 20)
    _say(f"[chunks] {many['n_chunks']}")
    assert many["n_chunks"] > 1
    np.testing.assert_array_equal(one["e_atom"], many["e_atom"])
    np.testing.assert_array_equal(one["forces"], many["forces"])


def test_fp32_deterministic():
    hp, s = CASES["D_12mixed"]()
    w = weights_for(hp, 9)
    a = gpu_run(hp, w, s, "fp32")
    b = gpu_run(hp, w, s, "fp32")
    np.testing.assert_array_equal(a["forces"], b["forces"])
    np.testing.assert_array_equal(a["virial"], b["virial"])
    np.testing.assert_array_equal(a["e_struct"], b["e_struct"])


def test_fp32_full_B_sampled_atoms():
    from oracle import model as M
    hp = synth.load_hparams("B")
    s = synth.config_b()
    w = synth.draw_weights(M.param_layout(M.HParams.from_dict(hp)), synth.WEIGHT_SEEDS["B"])
    gpu = gpu_run(hp, w, s, "fp32")
    assert gpu["status"] == 0
    atoms = synth.subset_rows(s.n_atoms, 12, 101)
    ref = M.forces_subset(M.HParams.from_dict(hp), w, s, atoms)
    fr = np.linalg.norm(gpu["forces"][atoms] - ref["forces"]) / np.linalg.norm(ref["forces"])
    mu = np.asarray([0.0])
    er = np.abs(gpu["e_atom"][atoms] - ref["e_atom"]).max()
    _say(f"[fp32 B sample] force rel {fr:.2e}, max |dE_i| {er:.2e}")
    assert fr <= FP32_TOL
    assert er <= 1e-5 * np.abs(ref["e_atom"]).max()
    F = gpu["forces"]
    assert np.abs(F.sum(0)).max() < 1e-6 * np.abs(F).max() * np.sqrt(s.n_atoms)
