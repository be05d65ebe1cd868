"""Value pin of the oracle's equivariant branch.

The invariance, finite-difference and locality pins hold for any
equivariant contraction, and the pair-potential case switches the whole
tensor-product branch off.  Here the per-atom energies of small open
clusters are evaluated a second time by hand, with plain vector algebra
(dot and cross products of 3-vectors, explicit loops over edges and rows,
no Clebsch-Gordan tensors, no einsum and no code from ``oracle``), and must
equal ``oracle.model.energy_forces`` to 1e-12.

What the hand evaluation fixes (the Allegro reading of Methodology / Model
Training, l_max = 1 in full O(3)):

* environment embedding omega = W_env x, row n (l_max + 1) + l;
* Gamma_i = nbar^-1/2 sum over row i of omega[n, l] Y^l (Y^0 = 1,
  Y^1 = sqrt(3) u_hat);
* initial features V^0 = omega^1 (x) Y (the edge's own embedding);
* channelwise products with the unit-normalised real coupling: scalar x
  scalar, scalar x vector, vector . vector / sqrt(3) (l = 1 x 1 -> 0) and
  vector x vector / sqrt(2) (1 x 1 -> 1);
* path sets after backward pruning and their order, typed out below;
* s = the 0e paths' outputs, path-major and channel-minor;
* V^L = sum over the paths into an irrep of alpha[path, n] T, or in the
  dense reading of the mixing sum over the paths into an irrep and over
  the input channels k of A_path[n, k] T[k];
* latent MLP on [x | s] with SiLU after every layer, times the envelope,
  residual (x + x~) / sqrt 2;
* eps = W_E2 W_E1 x; E_i = sigma_Z escale sum_row eps + mu_Z.

Vectors are kept in Cartesian (x, y, z) order: the library's l = 1 order
(y, z, x) is a cyclic permutation, a proper rotation, so every scalar
(and so every energy) is the same in either order -- and the 1 x 1 -> 1
coupling, the cross product in (y, z, x) order, is the cross product in
(x, y, z) order.

alpha, sigma_Z, mu_Z, nbar and energy_scale are all drawn away from 1, so
a mis-indexed mixing weight, a wrong normalisation power (nbar^-1 for
nbar^-1/2), channel-major s, a missing residual factor or V^0 built from
another layer's omega each move the energies far beyond the tolerance.
"""

import math

import numpy as np
import pytest

import synth

SQ3 = math.sqrt(3.0)
SQ2 = math.sqrt(2.0)


# --------------------------------------------------------------------------
# inputs

def hparams(n_layers, mixing="path"):
    return dict(n_species=3, l_max=1, n_layers=n_layers, latent=8, channels=4,
                n_bessel=5, poly_p=6, twobody=[6, 8], latent_depth=2,
                edge_hidden=5, r_cut=3.6, avg_num_neighbors=2.7,
                energy_scale=1.3, mixing=mixing)


# Path lists after backward pruning, typed out by hand as (l1, p1, l2, l3, p3),
# in the order (l1, p1 [+ first], l2, l3, p3 [+ first]).
#
# Two layers: layer 2 (the last) keeps the paths into (0, +): from (0, +)
# with l2 = 0 and from (1, -) with l2 = 1 ((1, +) with l2 = 1 gives (0, -)).
# So layer 1 must provide (0, +) and (1, -); its (1, -) x 1 -> (1, +) path
# is pruned.
PATHS_2 = [
    [(0, 1, 0, 0, 1), (0, 1, 1, 1, -1), (1, -1, 0, 1, -1), (1, -1, 1, 0, 1)],
    [(0, 1, 0, 0, 1), (1, -1, 1, 0, 1)],
]
# Three layers: layer 3 again needs (0, +) and (1, -); layer 2 produces
# (1, -) also from (1, +) x 1 -> (1, -), so layer 1's (1, +) output (the
# cross product) survives.
PATHS_3 = [
    [(0, 1, 0, 0, 1), (0, 1, 1, 1, -1), (1, -1, 0, 1, -1), (1, -1, 1, 0, 1), (1, -1, 1, 1, 1)],
    [(0, 1, 0, 0, 1), (0, 1, 1, 1, -1), (1, 1, 1, 1, -1), (1, -1, 0, 1, -1), (1, -1, 1, 0, 1)],
    [(0, 1, 0, 0, 1), (1, -1, 1, 0, 1)],
]


def layout(hp, paths):
    """(name, shape) of every weight block in the flat vector, in order (the
    library's documented layout)."""
    S, w, c, nb = hp["n_species"], hp["latent"], hp["channels"], hp["n_bessel"]
    t0, t1 = hp["twobody"]
    out = [("twobody.0", (t0, 2 * S + nb)), ("twobody.1", (t1, t0))]
    NL = hp["n_layers"]
    for L in range(1, NL + 1):
        n0 = sum(1 for p in paths[L - 1] if (p[3], p[4]) == (0, 1))
        out.append((f"layer{L}.env", (2 * c, w)))
        out.append((f"layer{L}.latent.0", (w, w + n0 * c)))
        out.append((f"layer{L}.latent.1", (w, w)))
        if L < NL:
            if hp["mixing"] == "dense":
                out.append((f"layer{L}.mix", (len(paths[L - 1]) * c, c)))
            else:
                out.append((f"layer{L}.alpha", (len(paths[L - 1]), c)))
    out += [("edge.0", (hp["edge_hidden"], w)), ("edge.1", (1, hp["edge_hidden"])),
            ("species.scale", (S,)), ("species.shift", (S,))]
    return out


def draw(hp, paths, seed):
    """Weights with every block away from its default: matrices N(0, 1/fan_in),
    alpha ~ +-U(0.4, 1.6), sigma_Z ~ U(0.5, 2), mu_Z ~ N(0, 1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts, blocks = [], {}
    for name, shape in layout(hp, paths):
        n = int(np.prod(shape))
        if name.endswith(".alpha"):
            v = rng.uniform(0.4, 1.6, n) * rng.choice([-1.0, 1.0], n)
        elif name == "species.scale":
            v = rng.uniform(0.5, 2.0, n)
        elif name == "species.shift":
            v = rng.standard_normal(n)
        else:
            v = rng.standard_normal(n) / math.sqrt(shape[1])
        parts.append(v)
        blocks[name] = v.reshape(shape)
    return np.concatenate(parts), blocks


def open_cluster(seed, n=4):
    """n atoms in a ~3 A ball (all pairs at 1.1-3.5 A) plus one atom just
    inside the cutoff of atom 0 only, in an open box."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pts = []
    while len(pts) < n:
        p = rng.uniform(-1.6, 1.6, 3)
        if all(1.1 < np.linalg.norm(p - q) < 3.5 for q in pts):
            pts.append(p)
    far = pts[0] + np.array([3.45, 0.3, -0.2])
    pos = np.array(pts + [far])
    species = rng.integers(0, 3, pos.shape[0]).astype(np.int32)
    return synth.System(pos, species, np.eye(3)[None] * 50.0, np.zeros(1, np.uint8),
                        np.array([0, pos.shape[0]], np.int64), 3)


# --------------------------------------------------------------------------
# the hand evaluation

def silu(a):
    return a / (1.0 + np.exp(-a))


def envelope6(x):
    return 1.0 - 28.0 * x ** 6 + 48.0 * x ** 7 - 21.0 * x ** 8 if x < 1.0 else 0.0


def product(path, V, G):
    """T of one path for one channel: V is the input feature (float for l1 = 0,
    3-vector for l1 = 1), G = (Gamma^0, Gamma^1) of the channel."""
    l1, _, l2, l3, _ = path
    g = G[l2]
    if l1 == 0 and l2 == 0:
        return V * g
    if l1 == 0:            # scalar x vector -> vector
        return V * g
    if l2 == 0:            # vector x scalar -> vector
        return V * g
    if l3 == 0:            # vector . vector / sqrt 3
        return float(np.dot(V, g)) / SQ3
    return np.cross(V, g) / SQ2      # vector x vector / sqrt 2


def hand_energies(hp, paths, P, sysd):
    S, c, w = hp["n_species"], hp["channels"], hp["latent"]
    rc, nb = hp["r_cut"], hp["n_bessel"]
    pos, Z = sysd.pos, sysd.species
    N = pos.shape[0]
    edges = [(i, j) for i in range(N) for j in range(N)
             if i != j and np.linalg.norm(pos[j] - pos[i]) < rc]
    geo = []
    for (i, j) in edges:
        d_vec = pos[j] - pos[i]
        d = float(np.linalg.norm(d_vec))
        u = envelope6(d / rc)
        rho = np.array([math.sqrt(2.0 / rc) * math.sin(k * math.pi * d / rc) / d
                        for k in range(1, nb + 1)]) * u
        geo.append((d, u, rho, SQ3 * d_vec / d))
    # two-body MLP
    x = []
    for (i, j), (d, u, rho, Y1) in zip(edges, geo):
        z = np.concatenate([np.eye(S)[Z[i]], np.eye(S)[Z[j]], rho])
        h = silu(P["twobody.1"] @ silu(P["twobody.0"] @ z))
        x.append(u * h)
    inv = 1.0 / math.sqrt(hp["avg_num_neighbors"])
    V = None     # V[e][n] = {irrep: value}
    NL = hp["n_layers"]
    for L in range(1, NL + 1):
        omega = [P[f"layer{L}.env"] @ xe for xe in x]          # [e][2c]
        G = [[(0.0, np.zeros(3)) for _ in range(c)] for _ in range(N)]
        for e, (i, _) in enumerate(edges):
            Y1 = geo[e][3]
            for n in range(c):
                g0, g1 = G[i][n]
                G[i][n] = (g0 + omega[e][2 * n + 0], g1 + omega[e][2 * n + 1] * Y1)
        G = [[(inv * g0, inv * g1) for (g0, g1) in row] for row in G]
        if L == 1:
            V = [[{(0, 1): omega[e][2 * n], (1, -1): omega[e][2 * n + 1] * geo[e][3]}
                  for n in range(c)] for e in range(len(edges))]
        newx, newV = [], []
        for e, (i, _) in enumerate(edges):
            T = [[product(pi, V[e][n][(pi[0], pi[1])], G[i][n]) for n in range(c)]
                 for pi in paths[L - 1]]
            s = [T[k][n] for k, pi in enumerate(paths[L - 1]) if (pi[3], pi[4]) == (0, 1)
                 for n in range(c)]
            u = geo[e][1]
            h = np.concatenate([x[e], np.array(s)])
            h = silu(P[f"layer{L}.latent.1"] @ silu(P[f"layer{L}.latent.0"] @ h))
            newx.append((x[e] + u * h) / SQ2)
            if L < NL and hp["mixing"] == "dense":
                A = P[f"layer{L}.mix"]          # row k c + n, column m
                feats = []
                for n in range(c):
                    f = {}
                    for k, pi in enumerate(paths[L - 1]):
                        key = (pi[3], pi[4])
                        for m in range(c):
                            f[key] = f.get(key, 0.0) + A[k * c + n, m] * T[k][m]
                    feats.append(f)
                newV.append(feats)
            elif L < NL:
                al = P[f"layer{L}.alpha"]
                feats = []
                for n in range(c):
                    f = {}
                    for k, pi in enumerate(paths[L - 1]):
                        key = (pi[3], pi[4])
                        f[key] = f.get(key, 0.0) + al[k, n] * T[k][n]
                    feats.append(f)
                newV.append(feats)
        x, V = newx, newV
    eps = [float((P["edge.1"] @ (P["edge.0"] @ xe))[0]) for xe in x]
    E = np.zeros(N)
    for e, (i, _) in enumerate(edges):
        E[i] += eps[e]
    zs = np.asarray(Z)
    return P["species.scale"][zs] * hp["energy_scale"] * E + P["species.shift"][zs]


# --------------------------------------------------------------------------

@pytest.mark.parametrize("n_layers,paths", [(2, PATHS_2), (3, PATHS_3)])
def test_path_lists_typed_by_hand(n_layers, paths):
    from oracle import model as M
    ps, _, _ = M.path_sets(M.HParams.from_dict(hparams(n_layers)))
    assert ps == paths


@pytest.mark.parametrize("mixing", ["path", "dense"])
@pytest.mark.parametrize("n_layers,paths", [(2, PATHS_2), (3, PATHS_3)])
@pytest.mark.parametrize("seed", [11, 12])
def test_energies_equal_hand_evaluation(n_layers, paths, seed, mixing):
    from oracle import model as M
    hp = hparams(n_layers, mixing)
    w, P = draw(hp, paths, 700 + seed)
    assert w.shape[0] == M.n_params(M.HParams.from_dict(hp))
    s = open_cluster(seed)
    ref = hand_energies(hp, paths, P, s)
    got = M.energy_forces(M.HParams.from_dict(hp), w, s, want_forces=False)["e_atom"]
    mu = P["species.shift"][s.species]
    # the branch must matter: the non-constant part is O(1) eV
    assert np.max(np.abs(ref - mu)) > 0.05
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12)


def test_hand_evaluation_sees_the_tensor_branch():
    """The value pin is only a pin of the branch if zeroing the tensor-product
    inputs s moves the energies by far more than the 1e-12 tolerance:
    compare with the hand model whose latent weights on s are zeroed."""
    hp = hparams(2)
    _, P = draw(hp, PATHS_2, 711)
    s = open_cluster(11)
    e_full = hand_energies(hp, PATHS_2, P, s)
    Q = dict(P)
    for L in (1, 2):
        W0 = P[f"layer{L}.latent.0"].copy()
        W0[:, hp["latent"]:] = 0.0
        Q[f"layer{L}.latent.0"] = W0
    e_cut = hand_energies(hp, PATHS_2, Q, s)
    assert np.max(np.abs(e_full - e_cut)) > 1e-4


def test_dense_mixing_is_seen():
    """The dense reading's pin is only a pin if the mixing matrices matter:
    transposing every A (a plausible index mistake) moves the energies far
    beyond the 1e-12 tolerance."""
    hp = hparams(3, "dense")
    _, P = draw(hp, PATHS_3, 733)
    s = open_cluster(12)
    e_ref = hand_energies(hp, PATHS_3, P, s)
    Q = dict(P)
    c = hp["channels"]
    for L in (1, 2):
        A = P[f"layer{L}.mix"].reshape(-1, c, c)
        Q[f"layer{L}.mix"] = np.ascontiguousarray(A.transpose(0, 2, 1)).reshape(-1, c)
    e_t = hand_energies(hp, PATHS_3, Q, s)
    assert np.max(np.abs(e_ref - e_t)) > 1e-4
