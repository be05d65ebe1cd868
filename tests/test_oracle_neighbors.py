"""Pins of the oracle neighbour lists: lattice-shell counts, agreement of the
two independent enumerations, reverse-edge symmetry, image handling."""

import dataclasses

import numpy as np
import pytest

import synth
from oracle import neighbors as nb


def _lattice(n, a, jitter=0.0, seed=5):
    return synth.cubic_lattice(n, a, jitter, 2, seed) if jitter else \
        dataclasses.replace(synth.cubic_lattice(n, a, 1e-300, 2, seed),
                            pos=synth.cubic_lattice(n, a, 1e-300, 2, seed).pos * 0
                            + np.stack(np.meshgrid(*(np.arange(n) * a,) * 3,
                                                   indexing="ij"), -1).reshape(-1, 3))


@pytest.mark.parametrize("a,r,count", [(2.2, 5.5, 80), (2.3, 5.5, 56),
                                       (2.3, 6.0, 80)])
def test_lattice_shell_counts(a, r, count):
    # shells n^2 = 1..6 hold 6, 12, 8, 6, 24, 24 sites
    s = _lattice(10, a)
    nl = nb.build(s, r, method="binned")
    deg = np.diff(nl["row_ptr"])
    assert np.all(deg == count)
    small = _lattice(4, a)           # 4 cells: brute force with images
    nl2 = nb.build(small, r, method="brute")
    assert np.all(np.diff(nl2["row_ptr"]) == count)


def test_binned_equals_brute_force_bitwise():
    s = synth.cubic_lattice(7, 2.2, 0.25, 3, 42)    # 15.4 A box, r = 5.0 -> 3 bins
    a = nb.build(s, 5.0, method="binned")
    b = nb.build(s, 5.0, method="brute")
    for k in ("i", "j", "n", "row_ptr", "rev"):
        np.testing.assert_array_equal(a[k], b[k])


def test_binned_handles_unwrapped_positions():
    s = synth.cubic_lattice(7, 2.2, 0.25, 3, 43)
    h = s.cell[0]
    rng = np.random.default_rng(0)
    k = rng.integers(-2, 3, size=(s.n_atoms, 3))
    moved = dataclasses.replace(s, pos=s.pos + nb.shift_vectors(h, k))
    a = nb.build(moved, 5.0, method="binned")
    b = nb.build(moved, 5.0, method="brute")
    for key in ("i", "j", "n", "row_ptr"):
        np.testing.assert_array_equal(a[key], b[key])
    # the same physical pairs as the wrapped system (n shifted by k_i - k_j)
    w = nb.build(s, 5.0, method="brute")
    np.testing.assert_array_equal(a["row_ptr"], w["row_ptr"])
    np.testing.assert_array_equal(a["j"], w["j"])


def test_reverse_edges_and_exact_antisymmetry():
    s = synth.config_a()
    nl = nb.build(s, 4.0)
    rev = nl["rev"]
    assert np.all(rev >= 0)
    np.testing.assert_array_equal(rev[rev], np.arange(rev.shape[0]))
    d = nb.edge_vectors(s, nl)
    np.testing.assert_array_equal(d[rev], -d)     # bit-exact negation


def test_canonical_order():
    s = synth.config_d(16)
    nl = nb.build(s, 6.0)
    key = np.lexsort((nl["n"][:, 2], nl["n"][:, 1], nl["n"][:, 0], nl["j"],
                      nl["i"]))
    np.testing.assert_array_equal(key, np.arange(key.shape[0]))


def test_small_triclinic_images_complete():
    """Cells narrower than the cutoff: every image within r must be found;
    compare with a much wider image range."""
    s = synth.config_d(8).structure(0)            # 8-atom-ish periodic cell
    r = 6.0
    ref_i, ref_j, ref_n = [], [], []
    w = nb.perpendicular_widths(s.cell[0])
    R = int(np.ceil(r / w.min())) + 2
    rngs = np.arange(-R, R + 1)
    imgs = np.stack(np.meshgrid(rngs, rngs, rngs, indexing="ij"), -1).reshape(-1, 3)
    sh = nb.shift_vectors(s.cell[0], imgs)
    for i in range(s.n_atoms):
        for j in range(s.n_atoms):
            dl = (s.pos[j] - s.pos[i])[None] + sh
            d2 = (dl[:, 0] * dl[:, 0] + dl[:, 1] * dl[:, 1]) + dl[:, 2] * dl[:, 2]
            for k in np.nonzero(d2 < r * r)[0]:
                if i == j and not imgs[k].any():
                    continue
                ref_i.append(i)
                ref_j.append(j)
                ref_n.append(imgs[k])
    nl = nb.build(s, r)
    assert nl["i"].shape[0] == len(ref_i)
    np.testing.assert_array_equal(nl["j"], np.array(ref_j))
    np.testing.assert_array_equal(nl["n"], np.array(ref_n))
    assert np.any(nl["i"] == nl["j"])              # self-images present


def test_open_clusters_have_no_images_and_rows_subset():
    s = synth.clusters(3, 20, 40, 0.1, 0.9, 4, 11)
    nl = nb.build(s, 5.0)
    assert np.all(nl["n"] == 0)
    rows = np.array([0, 5, 30])
    part = nb.build(s, 5.0, rows=rows)
    for r_ in rows:
        a = nl["j"][nl["i"] == r_]
        b = part["j"][part["i"] == r_]
        np.testing.assert_array_equal(a, b)


def test_wrap_keeps_inside_atoms_bit_identical():
    s = synth.cubic_lattice(5, 2.2, 0.25, 2, 3)
    pos = s.pos.copy()
    pos[0] += s.cell[0][0] * 1.0 + 0.1
    moved = dataclasses.replace(s, pos=pos)
    w = nb.wrap_positions(moved)
    inside = np.ones(s.n_atoms, bool)
    inside[0] = False
    frac = s.pos @ np.linalg.inv(s.cell[0])
    inside &= np.all((frac >= 0) & (frac < 1), axis=1)
    np.testing.assert_array_equal(w[inside], pos[inside])
    f0 = w[0] @ np.linalg.inv(s.cell[0])
    assert np.all((f0 >= 0) & (f0 < 1))
