"""Pins of the oracle model: closed forms of the basis, Table 1 parameter
counts, O(3)/translation/permutation invariance, finite differences of
energy (forces), strain (virial) and loss (double backward), strict
locality, and the special case that reduces the model to a pair potential."""

import dataclasses
import math

import numpy as np
import pytest
import torch

import synth
from oracle import model as M
from oracle import neighbors as nb
from oracle import so3


def hp_of(name, **kw):
    d = dict(synth.CONFIGS[name])
    d.update(avg_num_neighbors=10.0, energy_scale=1.0)
    d.update(kw)
    return M.HParams.from_dict(d)


def small_hp(**kw):
    """l_max = 2, two layers, narrow widths: exercises the 11 + 3 paths."""
    d = dict(n_species=3, l_max=2, n_layers=2, latent=16, channels=4,
             n_bessel=8, poly_p=6, twobody=[8, 16], latent_depth=2,
             edge_hidden=8, r_cut=4.0, avg_num_neighbors=8.0,
             energy_scale=1.0)
    d.update(kw)
    return M.HParams.from_dict(d)


def weights(hp, seed=5):
    w = synth.draw_weights(M.param_layout(hp), seed)
    return w


def cluster(n=14, seed=3, species=3):
    return synth.clusters(1, n, n, 0.1, 0.9, species, seed)


# ------------------------------------------------------------------ basis

def test_envelope_values_and_derivatives_at_ends():
    for p in (5, 6, 7):
        x = torch.tensor([0.0, 1.0 - 1e-12], dtype=torch.float64,
                         requires_grad=True)
        u = M.envelope(x, p)
        (g,) = torch.autograd.grad(u.sum(), x, create_graph=True)
        (h,) = torch.autograd.grad(g.sum(), x)
        assert abs(u[0].item() - 1.0) < 1e-15
        assert abs(u[1].item()) < 1e-9
        assert abs(g[1].item()) < 1e-8 and abs(h[1].item()) < 1e-6
        # p = 6: the DimeNet polynomial 1 - 28x^6 + 48x^7 - 21x^8
    xs = torch.linspace(0, 0.999, 50, dtype=torch.float64)
    ref = 1 - 28 * xs ** 6 + 48 * xs ** 7 - 21 * xs ** 8
    torch.testing.assert_close(M.envelope(xs, 6), ref, rtol=0, atol=1e-14)
    assert torch.all(M.envelope(torch.tensor([1.0, 1.3], dtype=torch.float64),
                                6) == 0)


def test_bessel_closed_form_and_limit():
    rc = 5.0
    d = torch.tensor([1e-7, 1.3, 4.9], dtype=torch.float64)
    B = M.bessel(d, rc, 8)
    for k, dd in enumerate([1e-7, 1.3, 4.9]):
        for n in range(1, 9):
            ref = math.sqrt(2 / rc) * math.sin(n * math.pi * dd / rc) / dd
            assert abs(B[k, n - 1].item() - ref) < 1e-12 * max(1, abs(ref))
    # d -> 0 limit sqrt(2/rc) n pi / rc
    np.testing.assert_allclose(B[0].numpy(), math.sqrt(2 / rc) * np.arange(1, 9)
                               * math.pi / rc, rtol=1e-10)


# ------------------------------------------------------------- structure

def test_table1_parameter_counts():
    """Table 1: 44.4K / 690K / 2.6M for FM64 / FM256 / FM512 (89 species,
    2 layers, l = 2, 8 Bessel functions).  The reading lands within
    -2%..+6%; the exact derived counts are pinned too."""
    paper = {64: 44.4e3, 256: 690e3, 512: 2.6e6}
    exact = {64: 46914, 256: 676466, 512: 2614194}
    for w, c, h in [(64, 16, 64), (256, 64, 128), (512, 128, 128)]:
        hp = M.HParams(89, 2, 2, w, c, 8, 6, [w // 4, w // 2, w], 3, h, 5.2)
        n = M.n_params(hp)
        assert n == exact[w]
        assert -0.02 <= n / paper[w] - 1 <= 0.06


def test_workload_parameter_counts_and_paths():
    want = {"A": (4836, [2]), "B": (665416, [11, 3]), "C": (175476, [11, 3]),
            "D": (972594, [15, 15, 3]), "E": (961544, [15, 15, 3])}
    for k, (n, paths) in want.items():
        hp = hp_of(k)
        assert M.n_params(hp) == n
        assert [len(p) for p in M.path_sets(hp)[0]] == paths


def test_sh_torch_matches_scipy_up_to_l3():
    """The model's torch harmonics against scipy's complex Y_lm (converted to
    the real, phase-free, component-normalised convention)."""
    import scipy.special as sps
    rng = np.random.default_rng(21)
    u = rng.standard_normal((60, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    th, ph = np.arccos(u[:, 2]), np.arctan2(u[:, 1], u[:, 0])
    for l in range(4):
        ref = []
        for m in range(-l, l + 1):
            Y = sps.sph_harm_y(l, abs(m), th, ph) * math.sqrt(4 * math.pi)
            ref.append(Y.real if m == 0 else math.sqrt(2) * (-1) ** m * (Y.real if m > 0 else Y.imag))
        got = M.sh_torch(l, torch.tensor(u, dtype=torch.float64)).numpy()
        np.testing.assert_allclose(got, np.stack(ref, 1), atol=1e-12)


def test_lmax3_path_counts_and_parities():
    """l_max = 3 in full O(3): 34 + 34 + 4 paths over three layers (23 + 4
    over two), four scalar paths per layer, every path parity-consistent."""
    for n_layers, counts in ((3, [34, 34, 4]), (2, [23, 4])):
        hp = small_hp(l_max=3, n_layers=n_layers)
        paths, ins, outs = M.path_sets(hp)
        assert [len(p) for p in paths] == counts
        assert [M.n_scalar_paths(p) for p in paths] == [4] * n_layers
        for L, ps in enumerate(paths):
            for (l1, p1, l2, l3, p3) in ps:
                assert p3 == p1 * (-1) ** l2 and abs(l1 - l2) <= l3 <= min(l1 + l2, 3)
                assert (l1, p1) in ins[L]


def test_path_parities():
    hp = hp_of("E")
    paths, ins, outs = M.path_sets(hp)
    for L, ps in enumerate(paths):
        for (l1, p1, l2, l3, p3) in ps:
            assert p3 == p1 * (-1) ** l2
            assert abs(l1 - l2) <= l3 <= l1 + l2 <= 4
            assert (l1, p1) in ins[L]
    assert all((p[3], p[4]) == (0, 1) for p in paths[-1])


# ------------------------------------------------------------ symmetries

def _energy(hp, w, s):
    return M.energy_forces(hp, w, s)


def test_invariances_and_equivariance_cluster():
    hp = small_hp()
    w = weights(hp)
    s = cluster()
    base = _energy(hp, w, s)
    rng = np.random.default_rng(0)
    Q = so3.random_rotation(rng)
    for R in (Q, -Q):                                   # rotation, rotoreflection
        t = rng.standard_normal(3) * 5
        s2 = dataclasses.replace(s, pos=s.pos @ R.T + t)
        r2 = _energy(hp, w, s2)
        np.testing.assert_allclose(r2["e_struct"], base["e_struct"], rtol=1e-12)
        np.testing.assert_allclose(r2["e_atom"], base["e_atom"], rtol=1e-11,
                                   atol=1e-12)
        np.testing.assert_allclose(r2["forces"], base["forces"] @ R.T,
                                   atol=1e-11)
    perm = rng.permutation(s.n_atoms)
    s3 = dataclasses.replace(s, pos=s.pos[perm], species=s.species[perm])
    r3 = _energy(hp, w, s3)
    np.testing.assert_allclose(r3["e_atom"], base["e_atom"][perm], rtol=1e-12)
    np.testing.assert_allclose(r3["forces"], base["forces"][perm], atol=1e-12)
    F = base["forces"]
    np.testing.assert_allclose(F.sum(0), 0, atol=1e-12)
    np.testing.assert_allclose(np.cross(s.pos, F).sum(0), 0, atol=1e-10)
    Wv = base["virial"][0]
    np.testing.assert_allclose(Wv, Wv.T, atol=1e-11)


def test_invariances_and_equivariance_lmax3():
    """The same symmetries with l_max = 3 (rotation and rotoreflection of a
    cluster, translation, permutation)."""
    hp = small_hp(l_max=3)
    w = weights(hp, 7)
    s = cluster(12, 5)
    base = _energy(hp, w, s)
    rng = np.random.default_rng(8)
    Q = so3.random_rotation(rng)
    for R in (Q, -Q):
        s2 = dataclasses.replace(s, pos=s.pos @ R.T + rng.standard_normal(3))
        r2 = _energy(hp, w, s2)
        np.testing.assert_allclose(r2["e_atom"], base["e_atom"], rtol=1e-11, atol=1e-12)
        np.testing.assert_allclose(r2["forces"], base["forces"] @ R.T, atol=1e-11)
    perm = rng.permutation(s.n_atoms)
    r3 = _energy(hp, w, dataclasses.replace(s, pos=s.pos[perm], species=s.species[perm]))
    np.testing.assert_allclose(r3["e_atom"], base["e_atom"][perm], rtol=1e-12)
    np.testing.assert_allclose(base["forces"].sum(0), 0, atol=1e-12)


def test_invariance_periodic_rotated_cell():
    hp = small_hp(r_cut=3.9, n_species=2)
    w = weights(hp)
    s = synth.config_a()
    base = _energy(hp, w, s)
    Q = so3.random_rotation(np.random.default_rng(4))
    s2 = dataclasses.replace(s, pos=s.pos @ Q.T, cell=s.cell @ Q.T)
    r2 = _energy(hp, w, s2)
    np.testing.assert_allclose(r2["e_struct"], base["e_struct"], rtol=1e-12)
    np.testing.assert_allclose(r2["forces"], base["forces"] @ Q.T, atol=1e-11)
    np.testing.assert_allclose(r2["virial"][0], Q @ base["virial"][0] @ Q.T,
                               atol=1e-10)


# ------------------------------------------------------ finite differences

@pytest.mark.parametrize("name", ["A", "small", "small_lmax3"])
def test_forces_central_differences(name):
    if name == "A":
        hp = hp_of("A", avg_num_neighbors=14.8)
        s = synth.config_a()
    else:
        hp = small_hp(l_max=3) if name == "small_lmax3" else small_hp()
        s = synth.config_a()
        s = dataclasses.replace(s, n_species=3)
    w = weights(hp)
    res = _energy(hp, w, s)
    h = 1e-5
    rng = np.random.default_rng(1)
    for a in rng.choice(s.n_atoms, 6, replace=False):
        for k in range(3):
            p = s.pos.copy()
            p[a, k] += h
            ep = M.energy_forces(hp, w, dataclasses.replace(s, pos=p),
                                 want_forces=False)["e_struct"][0]
            p[a, k] -= 2 * h
            em = M.energy_forces(hp, w, dataclasses.replace(s, pos=p),
                                 want_forces=False)["e_struct"][0]
            fd = -(ep - em) / (2 * h)
            assert abs(fd - res["forces"][a, k]) <= 1e-7 * max(
                1.0, np.abs(res["forces"]).max())


def test_virial_strain_differences():
    hp = hp_of("A", avg_num_neighbors=14.8)
    s = synth.config_a()
    w = weights(hp)
    res = _energy(hp, w, s)
    h = 1e-6
    for a in range(3):
        for b in range(3):
            es = []
            for sgn in (1, -1):
                eps = np.zeros((3, 3))
                eps[a, b] = sgn * h
                A = np.eye(3) + eps
                s2 = dataclasses.replace(s, pos=s.pos @ A.T, cell=s.cell @ A.T)
                es.append(M.energy_forces(hp, w, s2, want_forces=False)
                          ["e_struct"][0])
            fd = -(es[0] - es[1]) / (2 * h)
            assert abs(fd - res["virial"][0, a, b]) < 1e-6 * max(
                1.0, abs(res["virial"][0, a, b]))


def test_loss_gradient_finite_differences():
    hp = small_hp()
    s = synth.clusters(2, 8, 12, 0.1, 0.9, 3, 21)
    w = weights(hp, 8)
    e_hat, f_hat = synth.training_targets(s, 4)
    res = M.loss_and_grad(hp, w, s, e_hat, f_hat)
    g = res["grad_weights"]
    rng = np.random.default_rng(2)
    for _ in range(3):
        v = rng.standard_normal(w.shape[0])
        h = 1e-6
        lp = M.loss_and_grad(hp, w + h * v, s, e_hat, f_hat)["loss"]
        lm = M.loss_and_grad(hp, w - h * v, s, e_hat, f_hat)["loss"]
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g @ v) <= 1e-6 * max(abs(fd), 1e-3)


def test_vjp_weights_matches_loss_gradient_and_pos():
    """The generic double-backward entry reproduces the loss gradient, and its
    position derivative matches finite differences."""
    hp = small_hp()
    s = synth.clusters(1, 10, 10, 0.1, 0.9, 3, 23)
    w = weights(hp, 9)
    rng = np.random.default_rng(5)
    gE = rng.standard_normal(1)
    gF = rng.standard_normal((s.n_atoms, 3))
    out = M.vjp_weights(hp, w, s, gE, gF, want_pos=True)

    def obj(pos):
        r = M.energy_forces(hp, w, dataclasses.replace(s, pos=pos))
        return gE[0] * r["e_struct"][0] + np.sum(gF * r["forces"])

    h = 1e-5
    for a, k in [(0, 0), (4, 2), (9, 1)]:
        p = s.pos.copy()
        p[a, k] += h
        fp = obj(p)
        p[a, k] -= 2 * h
        fm = obj(p)
        assert abs((fp - fm) / (2 * h) - out["grad_pos"][a, k]) < 1e-6


# ------------------------------------------------------------- locality

def test_strict_locality_and_additivity():
    hp = small_hp()
    w = weights(hp)
    a = cluster(10, 31)
    b = cluster(12, 32)
    far = dataclasses.replace(b, pos=b.pos + np.array([100.0, 0, 0]))
    joint = dataclasses.replace(
        a, pos=np.concatenate([a.pos, far.pos]),
        species=np.concatenate([a.species, far.species]),
        seg=np.array([0, a.n_atoms + b.n_atoms]))
    ea = _energy(hp, w, a)["e_struct"][0]
    eb = _energy(hp, w, b)["e_struct"][0]
    ej = _energy(hp, w, joint)["e_struct"][0]
    assert abs(ej - (ea + eb)) < 1e-11 * abs(ej)
    # move an atom outside the cutoff ball of atom 0: E_0 unchanged
    res = _energy(hp, w, a)
    d = np.linalg.norm(a.pos - a.pos[0], axis=1)
    k = int(np.argmax(d))
    if d[k] > hp.r_cut + 0.5:
        p = a.pos.copy()
        p[k] += 0.2 * (p[k] - p[0]) / d[k]
        r2 = _energy(hp, w, dataclasses.replace(a, pos=p))
        assert r2["e_atom"][0] == pytest.approx(res["e_atom"][0], rel=1e-14)


def test_dimer_beyond_cutoff_is_sum_of_shifts():
    hp = small_hp()
    w = weights(hp)
    P = M.unpack(hp, torch.tensor(w))
    mu = P["species.shift"].numpy()
    for d in (hp.r_cut, hp.r_cut + 0.3):
        s = synth.System(np.array([[0, 0, 0], [d, 0, 0]], float),
                         np.array([0, 2], np.int32), np.zeros((1, 3, 3)),
                         np.zeros(1, np.uint8), np.array([0, 2]), 3)
        r = _energy(hp, w, s)
        assert r["e_struct"][0] == pytest.approx(mu[0] + mu[2], abs=1e-14)


def _silu(a):
    return a / (1 + np.exp(-a))


def test_pair_potential_special_case():
    """All W_env = 0 => Gamma = 0, V = 0, T = 0, s = 0: each edge energy is a
    function of (Z_i, Z_j, d) only.  Evaluated here directly in numpy."""
    hp = small_hp()
    w = weights(hp)
    lay = M.param_layout(hp)
    off = 0
    mats = {}
    for b in lay:
        if b["name"].endswith(".env"):
            w[off:off + b["size"]] = 0.0
        mats[b["name"]] = w[off:off + b["size"]].reshape(b["shape"])
        off += b["size"]
    s = synth.System(np.array([[0, 0, 0], [1.7, 0.4, -0.3]], float),
                     np.array([1, 2], np.int32), np.zeros((1, 3, 3)),
                     np.zeros(1, np.uint8), np.array([0, 2]), 3)
    r = _energy(hp, w, s)

    def eps(zi, zj, dd):
        x = dd / hp.r_cut
        u = 1 - 28 * x ** 6 + 48 * x ** 7 - 21 * x ** 8
        n = np.arange(1, 9)
        rho = math.sqrt(2 / hp.r_cut) * np.sin(n * math.pi * x) / dd * u
        z = np.concatenate([np.eye(3)[zi], np.eye(3)[zj], rho])
        h = z
        for k in range(2):
            h = _silu(mats[f"twobody.{k}"] @ h)
        xx = u * h
        for L in (1, 2):
            n0 = 3 if L == 1 else 3
            hin = np.concatenate([xx, np.zeros(n0 * hp.channels)])
            h = hin
            for k in range(2):
                h = _silu(mats[f"layer{L}.latent.{k}"] @ h)
            xx = (xx + u * h) / math.sqrt(2)
        return (mats["edge.1"] @ (mats["edge.0"] @ xx))[0]

    dd = np.linalg.norm(s.pos[1] - s.pos[0])
    e0 = eps(1, 2, dd) + mats["species.shift"][1]
    e1 = eps(2, 1, dd) + mats["species.shift"][2]
    np.testing.assert_allclose(r["e_atom"], [e0, e1], rtol=1e-12)
    # 1-D finite difference of the pair energy along the bond
    h = 1e-6
    fd = ((eps(1, 2, dd + h) + eps(2, 1, dd + h))
          - (eps(1, 2, dd - h) + eps(2, 1, dd - h))) / (2 * h)
    uvec = (s.pos[1] - s.pos[0]) / dd
    np.testing.assert_allclose(r["forces"][1], -fd * uvec, rtol=1e-7, atol=1e-10)


def test_lmax0_reduces_to_scalar_products():
    """l_max = 0: one path (0e x 0e -> 0e) with C = 1, so T = V * Gamma."""
    hp = small_hp(l_max=0, n_layers=1)
    assert M.path_sets(hp)[0] == [[(0, 1, 0, 0, 1)]]
    w = weights(hp)
    s = cluster(8, 41)
    r = _energy(hp, w, s)
    np.testing.assert_allclose(r["forces"].sum(0), 0, atol=1e-12)


def test_subset_forces_match_full():
    hp = small_hp()
    w = weights(hp)
    s = synth.cubic_lattice(5, 2.0, 0.2, 3, 9)
    full = _energy(hp, w, s)
    atoms = np.array([0, 17, 63, 124])
    sub = M.forces_subset(hp, w, s, atoms)
    np.testing.assert_allclose(sub["forces"], full["forces"][atoms], atol=1e-12)
    np.testing.assert_allclose(sub["e_atom"], full["e_atom"][atoms], rtol=1e-13)


def test_stress_loss_gradient_finite_differences():
    """Energy/force/stress loss (weights 8:1:1) on a batch with periodic and
    open structures: the double backward through the virial matches central
    differences of the loss in random weight directions."""
    hp = small_hp()
    s = synth.mixed_batch(3, 8, 12, 0.1, 3, 41)
    w = weights(hp, 10)
    e_hat, f_hat = synth.training_targets(s, 6)
    s_hat = synth.stress_targets(s, 7)
    res = M.loss_and_grad(hp, w, s, e_hat, f_hat, s_hat=s_hat, weights_efs=(8.0, 1.0, 1.0))
    assert res["grad_virial"] is not None and np.abs(res["grad_virial"][1]).max() == 0.0
    g = res["grad_weights"]
    rng = np.random.default_rng(3)
    for _ in range(3):
        v = rng.standard_normal(w.shape[0])
        h = 1e-6
        lp = M.loss_and_grad(hp, w + h * v, s, e_hat, f_hat, s_hat=s_hat, weights_efs=(8.0, 1.0, 1.0))["loss"]
        lm = M.loss_and_grad(hp, w - h * v, s, e_hat, f_hat, s_hat=s_hat, weights_efs=(8.0, 1.0, 1.0))["loss"]
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g @ v) <= 1e-6 * max(abs(fd), 1e-3)


def test_virial_term_of_the_double_backward_alone():
    """d/dtheta (gW : W) from the double backward equals central differences
    of gW : W, with W from the first-order oracle (pinned by strain FD)."""
    hp = small_hp()
    s = synth.mixed_batch(2, 9, 9, 0.1, 3, 43)
    w = weights(hp, 11)
    rng = np.random.default_rng(4)
    gW = rng.standard_normal((s.n_struct, 3, 3))
    out = M.vjp_weights(hp, w, s, np.zeros(s.n_struct), np.zeros((s.n_atoms, 3)), grad_virial=gW)
    v = rng.standard_normal(w.shape[0])
    h = 1e-6

    def obj(wv):
        return float(np.sum(gW * M.energy_forces(hp, wv, s)["virial"]))
    fd = (obj(w + h * v) - obj(w - h * v)) / (2 * h)
    assert abs(fd - out["grad_weights"] @ v) <= 1e-6 * max(abs(fd), 1e-3)


# ------------------------------------------------------ dense channel mixing

def _dense_from_alpha(hp_path, w_path, hp_dense):
    """The dense reading's weight vector whose mixing matrices are diag(alpha)
    of the path reading's vector (every other block copied)."""
    src = {b["name"]: b for b in M.param_layout(hp_path)}
    off, o = {}, 0
    for b in M.param_layout(hp_path):
        off[b["name"]] = o
        o += b["size"]
    out = []
    c = hp_dense.channels
    for b in M.param_layout(hp_dense):
        if b["name"].endswith(".mix"):
            a = src[b["name"][:-4] + ".alpha"]
            al = w_path[off[a["name"]]:off[a["name"]] + a["size"]].reshape(a["shape"])
            A = np.zeros((al.shape[0], c, c))
            for k in range(al.shape[0]):
                A[k] = np.diag(al[k])
            out.append(A.reshape(-1))
        else:
            out.append(w_path[off[b["name"]]:off[b["name"]] + b["size"]])
    return np.concatenate(out)


@pytest.mark.parametrize("lmax,nl", [(1, 3), (2, 2), (2, 3)])
def test_dense_mixing_with_diagonal_matrices_is_the_path_reading(lmax, nl):
    """A_pi = diag(alpha_pi) turns the dense reading into the per-path one:
    energies, forces and virial agree to rounding."""
    hp_p = small_hp(l_max=lmax, n_layers=nl)
    hp_d = small_hp(l_max=lmax, n_layers=nl, mixing="dense")
    w = weights(hp_p, 9)
    # alpha away from 1 so the diagonal carries information
    rng = np.random.default_rng(3)
    o = 0
    for b in M.param_layout(hp_p):
        if b["name"].endswith(".alpha"):
            w[o:o + b["size"]] = rng.uniform(0.4, 1.6, b["size"]) * rng.choice([-1, 1], b["size"])
        o += b["size"]
    wd = _dense_from_alpha(hp_p, w, hp_d)
    assert wd.shape[0] == M.n_params(hp_d)
    s = synth.config_a()
    s = dataclasses.replace(s, n_species=3)
    rp = M.energy_forces(hp_p, w, s)
    rd = M.energy_forces(hp_d, wd, s)
    np.testing.assert_allclose(rd["e_atom"], rp["e_atom"], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(rd["forces"], rp["forces"], rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(rd["virial"], rp["virial"], rtol=1e-11, atol=1e-10)


def test_dense_mixing_parameter_count():
    """The dense reading replaces each alpha [n_paths, c] by n_paths c x c
    matrices: Table 1's FM64 / FM256 / FM512 shapes then have
    49.6K / 720.8K / 2.79M weights, further from the paper's 44.4K / 690K /
    2.6M than the per-path reading (the reason it is not the default)."""
    want = {64: (16, 64, 49554), 256: (64, 128, 720818), 512: (128, 128, 2793010)}
    for w_, (c, h, n) in want.items():
        d = dict(n_species=89, l_max=2, n_layers=2, latent=w_, channels=c, n_bessel=8, poly_p=6,
                 twobody=[w_ // 4, w_ // 2, w_], latent_depth=3, edge_hidden=h, r_cut=5.2)
        npd = M.n_params(M.HParams.from_dict(dict(d, mixing="dense")))
        npp = M.n_params(M.HParams.from_dict(d))
        paths, _, _ = M.path_sets(M.HParams.from_dict(d))
        assert npd - npp == len(paths[0]) * c * (c - 1)
        assert npd == n, (w_, npd)


def test_dense_mixing_invariances_and_force_differences():
    """Random dense mixing keeps O(3), translation and permutation invariance,
    and the forces are the energy's central differences."""
    hp = small_hp(n_layers=3, mixing="dense")
    w = weights(hp, 13)
    s = cluster(12, 6)
    base = _energy(hp, w, s)
    rng = np.random.default_rng(14)
    Q = so3.random_rotation(rng)
    for R in (Q, -Q):
        s2 = dataclasses.replace(s, pos=s.pos @ R.T + rng.standard_normal(3))
        r2 = _energy(hp, w, s2)
        np.testing.assert_allclose(r2["e_atom"], base["e_atom"], rtol=1e-11, atol=1e-12)
        np.testing.assert_allclose(r2["forces"], base["forces"] @ R.T, atol=1e-11)
    perm = rng.permutation(s.n_atoms)
    r3 = _energy(hp, w, dataclasses.replace(s, pos=s.pos[perm], species=s.species[perm]))
    np.testing.assert_allclose(r3["e_atom"], base["e_atom"][perm], rtol=1e-12)
    np.testing.assert_allclose(base["forces"].sum(0), 0, atol=1e-12)
    h = 1e-5
    for a in rng.choice(s.n_atoms, 4, replace=False):
        for k in range(3):
            p = s.pos.copy()
            p[a, k] += h
            ep = M.energy_forces(hp, w, dataclasses.replace(s, pos=p), want_forces=False)["e_struct"][0]
            p[a, k] -= 2 * h
            em = M.energy_forces(hp, w, dataclasses.replace(s, pos=p), want_forces=False)["e_struct"][0]
            fd = -(ep - em) / (2 * h)
            assert abs(fd - base["forces"][a, k]) <= 1e-7 * max(1.0, np.abs(base["forces"]).max())
