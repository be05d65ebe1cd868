"""Oracle model: energy, forces, virial, loss and weight gradients in float64
(test infrastructure only).

The paper (Methodology / Model Training; Table 1) trains Allegro with: a
two-body latent MLP on (species_i, species_j, radial basis), tensor features
with l up to 2 in full O(3), an embedding MLP that is a single linear
projection, latent MLPs with SiLU, an edge-energy MLP with one hidden layer and
no nonlinearity, and a radial cutoff.  Energies are per-atom sums of edge
energies; forces and stress are derivatives of the energy (they enter the
8:1:1 loss).  The architecture equations themselves are not printed; this
module follows the Allegro formulation with these readings:

  basis      x = d / r_c; u(x) = 1 - (p+1)(p+2)/2 x^p + p(p+2) x^(p+1)
             - p(p+1)/2 x^(p+2) for x < 1 else 0;
             B_n(d) = sqrt(2 / r_c) sin(n pi x) / d, n = 1..n_b; rho = B u.
  two-body   x0 = u * MLP_2b([onehot(Z_i) | onehot(Z_j) | rho]); SiLU after
             every layer including the last; no biases anywhere.
  layer L    omega = W_env^L x^(L-1), viewed as [c, l_max + 1];
             Gamma_i[n, l, m] = nbar^-1/2 sum_{e in row i} omega_e[n, l] Y^l_e[m];
             V^0_e[n, (l, (-1)^l), m] = omega^1_e[n, l] Y^l_e[m];
             T^pi_e[n, m3] = sum C[m1, m2, m3] V^(L-1)_e[n, ir1, m1]
                             * Gamma_i(e)[n, l2, m2]   (channelwise);
             s_e = T^pi_e[:, 0] over the 0e paths (path-major, channel-minor);
             x~ = u * MLP_lat([x^(L-1) | s_e]); x^L = (x^(L-1) + x~) / sqrt 2;
             V^L[n, ir3] = sum_{pi -> ir3} alpha^L[pi, n] T^pi[n]  (L < N_L);
             or, with mixing = "dense" (the alternative reading, a c x c
             channel-mixing matrix per path after the products):
             V^L[n, ir3] = sum_{pi -> ir3} sum_k A^L_pi[n, k] T^pi[k].
  energy     eps_e = W_E2 W_E1 x^(N_L);
             E_i = sigma_Z(i) * energy_scale * sum_{row i} eps_e + mu_Z(i);
             E_s = sum_{i in s} E_i.
  forces     g_e = dE/d delta_e (autograd);  F_i = sum_{e: i(e)=i} g_e
             - sum_{e: j(e)=i} g_e;  W_s = - sum_{e in s} g_e delta_e^T.

Paths: hidden irreps are every (l <= l_max, p = +-1); the last layer keeps
only (0, +) outputs; paths whose outputs are not consumed are pruned
backwards; order is lexicographic on (l1, p1 [+ first], l2, l3, p3 [+ first]).

Weight layout (flat float64 vector, row-major out x in matrices, in order):
  twobody.k [h_k+1, h_k] (h_0 = 2S + n_b), fan-in init;
  per layer: layer{L}.env [c (l_max+1), w]; layer{L}.latent.k (first has
  in = w + n0e c); layer{L}.alpha [n_paths, c] (ones; only L < N_L) or,
  dense mixing, layer{L}.mix [n_paths c, c] (row pi c + n, column k:
  A^L_pi[n, k]; fan-in c init; only L < N_L);
  edge.0 [h, w]; edge.1 [1, h]; species.scale [S] (ones);
  species.shift [S] (N(0, 1)).

Pins: invariances, finite differences, locality, the pair-potential special
case (all W_env = 0), Table 1's parameter counts, and a value pin of the
equivariant branch: per-atom energies of open clusters (l_max = 1, two and
three layers, alpha, sigma_Z, nbar and energy_scale away from 1) evaluated
independently with dot and cross products (tests/test_oracle_*); the
dense mixing reading by the same hand evaluation with explicit sums over
channels, by its reduction to the per-path reading when every A is
diagonal, and by invariance and finite differences with random A.
The match to the trained Allegro-FM models themselves is parity unpinned (no
weights or code exist).
"""

from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np
import torch

from . import neighbors as nbr
from . import so3

DT = torch.float64


@dataclasses.dataclass
class HParams:
    n_species: int
    l_max: int
    n_layers: int
    latent: int
    channels: int
    n_bessel: int
    poly_p: int
    twobody: List[int]
    latent_depth: int
    edge_hidden: int
    r_cut: float
    avg_num_neighbors: float = 1.0
    energy_scale: float = 1.0
    mixing: str = "path"        # "path" (alpha per path and channel) or "dense"

    @staticmethod
    def from_dict(d: Dict) -> "HParams":
        keys = {f.name for f in dataclasses.fields(HParams)}
        return HParams(**{k: v for k, v in d.items() if k in keys})


Irrep = Tuple[int, int]          # (l, p), p in {+1, -1}
Path = Tuple[int, int, int, int, int]   # (l1, p1, l2, l3, p3)


def _pkey(p: int) -> int:
    return 0 if p == 1 else 1


def irrep_sort_key(ir: Irrep):
    return (ir[0], _pkey(ir[1]))


def path_sort_key(pi: Path):
    l1, p1, l2, l3, p3 = pi
    return (l1, _pkey(p1), l2, l3, _pkey(p3))


def path_sets(hp: HParams):
    """Per-layer pruned path lists and the irreps of V^(L-1) each reads.

    Returns (paths, in_irreps, out_irreps): paths[L-1] is the sorted path list
    of layer L; in_irreps[L-1] the irreps of V^(L-1) that exist; out_irreps[L-1]
    the irreps of V^L (empty for the last layer)."""
    lm = hp.l_max
    NL = hp.n_layers
    avail: List[List[Irrep]] = [[(l, (-1) ** l) for l in range(lm + 1)]]
    full: List[List[Path]] = []
    for L in range(1, NL + 1):
        ps = []
        for (l1, p1) in avail[-1]:
            for l2 in range(lm + 1):
                for l3 in range(abs(l1 - l2), min(l1 + l2, lm) + 1):
                    p3 = p1 * (-1) ** l2
                    if L == NL and (l3, p3) != (0, 1):
                        continue
                    ps.append((l1, p1, l2, l3, p3))
        full.append(ps)
        avail.append(sorted({(p[3], p[4]) for p in ps}, key=irrep_sort_key))
    # backward pruning: keep outputs consumed by the next layer or 0e scalars
    for L in range(NL - 1, 0, -1):
        used_next = {(p[0], p[1]) for p in full[L]}
        full[L - 1] = [p for p in full[L - 1]
                       if (p[3], p[4]) in used_next or (p[3], p[4]) == (0, 1)]
    paths = [sorted(ps, key=path_sort_key) for ps in full]
    in_irreps = [avail[0]] + [sorted({(p[3], p[4]) for p in paths[L]},
                                     key=irrep_sort_key)
                              for L in range(NL - 1)]
    out_irreps = [in_irreps[L + 1] for L in range(NL - 1)] + [[]]
    return paths, in_irreps, out_irreps


def n_scalar_paths(paths: Sequence[Path]) -> int:
    return sum(1 for p in paths if (p[3], p[4]) == (0, 1))


def param_layout(hp: HParams) -> List[Dict]:
    """Ordered parameter blocks: name, shape, size, fan_in, init kind."""
    S, w, c, lm = hp.n_species, hp.latent, hp.channels, hp.l_max
    paths, _, _ = path_sets(hp)
    blocks = []

    def mat(name, out, inp, init="fan_in"):
        blocks.append(dict(name=name, shape=(out, inp), size=out * inp,
                           fan_in=inp, init=init))

    dims = [2 * S + hp.n_bessel] + list(hp.twobody)
    for k in range(len(hp.twobody)):
        mat(f"twobody.{k}", dims[k + 1], dims[k])
    if hp.twobody[-1] != w:
        raise ValueError("last two-body width must equal the latent width")
    for L in range(1, hp.n_layers + 1):
        mat(f"layer{L}.env", c * (lm + 1), w)
        n0 = n_scalar_paths(paths[L - 1])
        ind = w + n0 * c
        for k in range(hp.latent_depth):
            mat(f"layer{L}.latent.{k}", w, ind if k == 0 else w)
        if L < hp.n_layers:
            np_ = len(paths[L - 1])
            if hp.mixing == "dense":
                mat(f"layer{L}.mix", np_ * c, c)
            elif hp.mixing == "path":
                blocks.append(dict(name=f"layer{L}.alpha", shape=(np_, c),
                                   size=np_ * c, fan_in=1, init="ones"))
            else:
                raise ValueError(f"unknown mixing {hp.mixing!r}")
    mat("edge.0", hp.edge_hidden, w)
    mat("edge.1", 1, hp.edge_hidden)
    blocks.append(dict(name="species.scale", shape=(S,), size=S, fan_in=1,
                       init="ones"))
    blocks.append(dict(name="species.shift", shape=(S,), size=S, fan_in=1,
                       init="normal"))
    return blocks


def n_params(hp: HParams) -> int:
    return sum(b["size"] for b in param_layout(hp))


def unpack(hp: HParams, flat: torch.Tensor) -> Dict[str, torch.Tensor]:
    out = {}
    o = 0
    for b in param_layout(hp):
        out[b["name"]] = flat[o:o + b["size"]].view(*b["shape"])
        o += b["size"]
    if o != flat.shape[0]:
        raise ValueError(f"weight vector has {flat.shape[0]} values, layout {o}")
    return out


# --------------------------------------------------------------------------
# building blocks, each a plain transcription of its definition

def envelope(x: torch.Tensor, p: int) -> torch.Tensor:
    """Polynomial cutoff u(x), zero for x >= 1 (DimeNet form)."""
    poly = (1.0 - (p + 1) * (p + 2) / 2.0 * x ** p + p * (p + 2) * x ** (p + 1)
            - p * (p + 1) / 2.0 * x ** (p + 2))
    return torch.where(x < 1.0, poly, torch.zeros_like(x))


def bessel(d: torch.Tensor, r_c: float, n_b: int) -> torch.Tensor:
    """B_n(d) = sqrt(2 / r_c) sin(n pi d / r_c) / d, n = 1..n_b."""
    n = torch.arange(1, n_b + 1, dtype=DT)
    return math.sqrt(2.0 / r_c) * torch.sin(n[None, :] * math.pi * d[:, None]
                                            / r_c) / d[:, None]


def sh_torch(l: int, u: torch.Tensor) -> torch.Tensor:
    x, y, z = u[:, 0], u[:, 1], u[:, 2]
    if l == 0:
        return torch.ones_like(x)[:, None]
    if l == 1:
        return math.sqrt(3.0) * torch.stack([y, z, x], dim=1)
    if l == 2:
        s15 = math.sqrt(15.0)
        return torch.stack([s15 * x * y, s15 * y * z,
                            0.5 * math.sqrt(5.0) * (3.0 * z * z - 1.0),
                            s15 * x * z, 0.5 * s15 * (x * x - y * y)], dim=1)
    if l == 3:
        # the l = 3 real harmonics of the same convention (no Condon-Shortley
        # phase, sum_m Y^2 = 7), m = -3..3
        a3, a2, a1, a0 = math.sqrt(35.0 / 8.0), math.sqrt(105.0), math.sqrt(21.0 / 8.0), math.sqrt(7.0) / 2.0
        return torch.stack([a3 * y * (3.0 * x * x - y * y), a2 * x * y * z,
                            a1 * y * (5.0 * z * z - 1.0), a0 * z * (5.0 * z * z - 3.0),
                            a1 * x * (5.0 * z * z - 1.0), 0.5 * a2 * z * (x * x - y * y),
                            a3 * x * (x * x - 3.0 * y * y)], dim=1)
    raise ValueError("l_max <= 3 in the oracle model")


def silu(a: torch.Tensor) -> torch.Tensor:
    return a * torch.sigmoid(a)


def mlp(h: torch.Tensor, mats: Sequence[torch.Tensor]) -> torch.Tensor:
    for W in mats:
        h = silu(h @ W.T)
    return h


def cg_t(l1: int, l2: int, l3: int) -> torch.Tensor:
    return torch.tensor(np.array(so3.cg(l1, l2, l3)), dtype=DT)


def rows_energy(hp: HParams, P: Dict[str, torch.Tensor], delta: torch.Tensor,
                zi: torch.Tensor, zj: torch.Tensor, row: torch.Tensor,
                z_rows: torch.Tensor) -> torch.Tensor:
    """Per-atom energies E_i of `n_rows` central atoms from their edges.

    delta [E, 3], zi/zj [E] species of the central and neighbour atom, row [E]
    local row index in [0, n_rows), z_rows [n_rows] species of the rows.
    """
    n_rows = z_rows.shape[0]
    S, c, lm = hp.n_species, hp.channels, hp.l_max
    paths, in_irreps, _ = path_sets(hp)
    E = delta.shape[0]
    d = torch.sqrt((delta * delta).sum(dim=1))
    uhat = delta / d[:, None]
    u = envelope(d / hp.r_cut, hp.poly_p)
    rho = bessel(d, hp.r_cut, hp.n_bessel) * u[:, None]
    Y = [sh_torch(l, uhat) for l in range(lm + 1)]
    oh_i = torch.nn.functional.one_hot(zi, S).to(DT)
    oh_j = torch.nn.functional.one_hot(zj, S).to(DT)
    z0 = torch.cat([oh_i, oh_j, rho], dim=1)
    x = u[:, None] * mlp(z0, [P[f"twobody.{k}"] for k in range(len(hp.twobody))])
    inv_sqrt_nbar = 1.0 / math.sqrt(hp.avg_num_neighbors)
    V = None
    for L in range(1, hp.n_layers + 1):
        omega = (x @ P[f"layer{L}.env"].T).view(E, c, lm + 1)
        Gam = []
        for l in range(lm + 1):
            per_edge = omega[:, :, l, None] * Y[l][:, None, :]
            g = torch.zeros(n_rows, c, 2 * l + 1, dtype=DT)
            g = g.index_add(0, row, per_edge)
            Gam.append(inv_sqrt_nbar * g)
        if L == 1:
            V = {(l, (-1) ** l): omega[:, :, l, None] * Y[l][:, None, :]
                 for l in range(lm + 1)}
        T = []
        for (l1, p1, l2, l3, p3) in paths[L - 1]:
            C = cg_t(l1, l2, l3)
            Ge = Gam[l2][row]
            T.append(torch.einsum("abk,eca,ecb->eck", C, V[(l1, p1)], Ge))
        s = torch.cat([T[k][:, :, 0] for k, p in enumerate(paths[L - 1])
                       if (p[3], p[4]) == (0, 1)], dim=1)
        hin = torch.cat([x, s], dim=1)
        xt = u[:, None] * mlp(hin, [P[f"layer{L}.latent.{k}"]
                                    for k in range(hp.latent_depth)])
        x = (x + xt) / math.sqrt(2.0)
        if L < hp.n_layers:
            if hp.mixing == "dense":
                A = P[f"layer{L}.mix"].view(len(paths[L - 1]), c, c)
            else:
                alpha = P[f"layer{L}.alpha"]
            Vn = {}
            for k, (l1, p1, l2, l3, p3) in enumerate(paths[L - 1]):
                if hp.mixing == "dense":
                    term = torch.matmul(A[k], T[k])       # [c, c] @ [E, c, 2 l3 + 1]
                else:
                    term = alpha[k][None, :, None] * T[k]
                key = (l3, p3)
                Vn[key] = term if key not in Vn else Vn[key] + term
            V = Vn
    eps = (x @ P["edge.0"].T) @ P["edge.1"].T           # [E, 1]
    esum = torch.zeros(n_rows, dtype=DT).index_add(0, row, eps[:, 0])
    return (P["species.scale"][z_rows] * hp.energy_scale * esum
            + P["species.shift"][z_rows])


# --------------------------------------------------------------------------
# whole-batch drivers

def _as_hp(hp) -> HParams:
    return hp if isinstance(hp, HParams) else HParams.from_dict(hp)


def energy_forces(hp, weights: np.ndarray, sys, nl: Optional[Dict] = None,
                  r_list: Optional[float] = None, chunk: int = 512,
                  grad_e_struct: Optional[np.ndarray] = None,
                  want_forces: bool = True) -> Dict[str, np.ndarray]:
    """E_i, E_s, F, W (and g_e) of a whole batch in float64.

    Central atoms are processed in chunks (exact: E_i depends only on the edges
    of row i).  `grad_e_struct` weights the structures' energies for the
    derivative (defaults to ones).
    """
    hp = _as_hp(hp)
    if nl is None:
        nl = nbr.build(sys, hp.r_cut if r_list is None else r_list)
    W = torch.tensor(weights, dtype=DT)
    P = unpack(hp, W)
    delta_all = nbr.edge_vectors(sys, nl)
    N = sys.n_atoms
    I = nl["i"]
    J = nl["j"]
    row_ptr = nl["row_ptr"]
    species = torch.tensor(sys.species.astype(np.int64))
    struct_of_atom = np.searchsorted(sys.seg, np.arange(N), side="right") - 1
    ges = np.ones(sys.n_struct) if grad_e_struct is None else grad_e_struct
    e_atom = np.zeros(N)
    g_all = np.zeros_like(delta_all)
    for a in range(0, N, chunk):
        b = min(N, a + chunk)
        e0, e1 = int(row_ptr[a]), int(row_ptr[b])
        delta = torch.tensor(delta_all[e0:e1], dtype=DT,
                             requires_grad=want_forces)
        Ic = torch.tensor(I[e0:e1])
        Jc = torch.tensor(J[e0:e1])
        Ei = rows_energy(hp, P, delta, species[Ic], species[Jc], Ic - a,
                         species[a:b])
        e_atom[a:b] = Ei.detach().numpy()
        if want_forces and e1 > e0:
            wts = torch.tensor(ges[struct_of_atom[a:b]], dtype=DT)
            (g,) = torch.autograd.grad((Ei * wts).sum(), delta)
            g_all[e0:e1] = g.numpy()
    e_struct = np.array([e_atom[sys.seg[s]:sys.seg[s + 1]].sum()
                         for s in range(sys.n_struct)])
    out = dict(e_atom=e_atom, e_struct=e_struct, nl=nl, delta=delta_all)
    if want_forces:
        F = np.zeros((N, 3))
        np.add.at(F, I, g_all)
        np.add.at(F, J, -g_all)
        Wv = np.zeros((sys.n_struct, 3, 3))
        es = struct_of_atom[I]
        np.add.at(Wv, es, -g_all[:, :, None] * delta_all[:, None, :])
        out.update(forces=F, virial=Wv, g=g_all)
    return out


def forces_subset(hp, weights: np.ndarray, sys, atoms: np.ndarray,
                  r_list: Optional[float] = None) -> Dict[str, np.ndarray]:
    """Exact E_k and F_k for selected atoms k of a large batch.

    F_k needs every E_i whose row contains k: the rows {k} and N(k).  Only
    those rows' edges are built and evaluated.
    """
    hp = _as_hp(hp)
    r = hp.r_cut if r_list is None else r_list
    atoms = np.asarray(atoms, np.int64)
    nl_k = nbr.build(sys, r, rows=atoms)
    rows = np.unique(np.concatenate([atoms, nl_k["j"]]))
    nl = nbr.build(sys, r, rows=rows)
    W = torch.tensor(weights, dtype=DT)
    P = unpack(hp, W)
    delta_all = nbr.edge_vectors(sys, nl)
    species = torch.tensor(sys.species.astype(np.int64))
    g = np.zeros_like(delta_all)
    Ei_all = np.zeros(rows.shape[0])
    # rows are sorted and the list is row-major: chunks of rows are
    # contiguous edge ranges (exact by locality)
    rstart = np.searchsorted(nl["i"], rows, side="left")
    rend = np.searchsorted(nl["i"], rows, side="right")
    chunk = 256
    for c0 in range(0, rows.shape[0], chunk):
        c1 = min(rows.shape[0], c0 + chunk)
        e0, e1 = int(rstart[c0]), int(rend[c1 - 1])
        delta = torch.tensor(delta_all[e0:e1], dtype=DT, requires_grad=True)
        I = torch.tensor(nl["i"][e0:e1])
        J = torch.tensor(nl["j"][e0:e1])
        loc = torch.tensor(np.searchsorted(rows[c0:c1], nl["i"][e0:e1]))
        Ei = rows_energy(hp, P, delta, species[I], species[J], loc,
                         species[torch.tensor(rows[c0:c1])])
        Ei_all[c0:c1] = Ei.detach().numpy()
        if e1 > e0:
            (gc,) = torch.autograd.grad(Ei.sum(), delta)
            g[e0:e1] = gc.numpy()
    F = np.zeros((atoms.shape[0], 3))
    pos_of = {int(k): t for t, k in enumerate(atoms)}
    for e in range(g.shape[0]):
        t = pos_of.get(int(nl["i"][e]))
        if t is not None:
            F[t] += g[e]
        t = pos_of.get(int(nl["j"][e]))
        if t is not None:
            F[t] -= g[e]
    e_atoms = Ei_all[np.searchsorted(rows, atoms)]
    return dict(e_atom=e_atoms, forces=F, n_rows=rows.shape[0],
                n_edges=int(g.shape[0]))


def rows_energy_grad(hp, weights: np.ndarray, sys, rows: np.ndarray,
                     r_list: Optional[float] = None, chunk: int = 256) -> Dict[str, np.ndarray]:
    """E_i of the given central atoms and g_e = dE/d delta_e of their edges:
    the per-row share of one energy+force evaluation (rows are independent
    by locality).  Used to time the oracle on a bounded sample."""
    hp = _as_hp(hp)
    rows = np.sort(np.asarray(rows, np.int64))
    nl = nbr.build(sys, hp.r_cut if r_list is None else r_list, rows=rows)
    P = unpack(hp, torch.tensor(weights, dtype=DT))
    species = torch.tensor(sys.species.astype(np.int64))
    delta_all = nbr.edge_vectors(sys, nl)
    g = np.zeros_like(delta_all)
    E = np.zeros(rows.shape[0])
    rs = np.searchsorted(nl["i"], rows, side="left")
    re = np.searchsorted(nl["i"], rows, side="right")
    for c0 in range(0, rows.shape[0], chunk):
        c1 = min(rows.shape[0], c0 + chunk)
        e0, e1 = int(rs[c0]), int(re[c1 - 1])
        delta = torch.tensor(delta_all[e0:e1], dtype=DT, requires_grad=True)
        I = torch.tensor(nl["i"][e0:e1])
        J = torch.tensor(nl["j"][e0:e1])
        loc = torch.tensor(np.searchsorted(rows[c0:c1], nl["i"][e0:e1]))
        Ei = rows_energy(hp, P, delta, species[I], species[J], loc,
                         species[torch.tensor(rows[c0:c1])])
        E[c0:c1] = Ei.detach().numpy()
        if e1 > e0:
            (gc,) = torch.autograd.grad(Ei.sum(), delta)
            g[e0:e1] = gc.numpy()
    return dict(e_atom=E, g=g, n_edges=int(g.shape[0]))


def vjp_weights(hp, weights: np.ndarray, sys, grad_e_struct: np.ndarray,
                grad_forces: np.ndarray, nl: Optional[Dict] = None,
                r_list: Optional[float] = None,
                want_pos: bool = False,
                grad_virial: Optional[np.ndarray] = None) -> Dict[str, np.ndarray]:
    """d/dtheta [sum_s gE_s E_s + sum_i gF_i . F_i + sum_s gW_s : W_s] by
    double backward (float64 autograd with create_graph), one structure at a
    time (exact: structures do not interact), with the virial
    W_s = -sum_e g_e delta_e^T built inside the graph.  Optionally the same
    derivative with respect to the positions."""
    hp = _as_hp(hp)
    if nl is None:
        nl = nbr.build(sys, hp.r_cut if r_list is None else r_list)
    Wt = torch.tensor(weights, dtype=DT, requires_grad=True)
    P = unpack(hp, Wt)
    species = torch.tensor(sys.species.astype(np.int64))
    grad = torch.zeros_like(Wt)
    gpos = np.zeros((sys.n_atoms, 3))
    for s in range(sys.n_struct):
        a, b = int(sys.seg[s]), int(sys.seg[s + 1])
        e0, e1 = int(nl["row_ptr"][a]), int(nl["row_ptr"][b])
        pos = torch.tensor(sys.pos[a:b], dtype=DT, requires_grad=want_pos)
        Il = torch.tensor(nl["i"][e0:e1] - a)
        Jl = torch.tensor(nl["j"][e0:e1] - a)
        if sys.pbc[s]:
            sh = torch.tensor(nbr.shift_vectors(sys.cell[s], nl["n"][e0:e1]),
                              dtype=DT)
        else:
            sh = torch.zeros(e1 - e0, 3, dtype=DT)
        if want_pos:
            delta = (pos[Jl] - pos[Il]) + sh
        else:
            delta = torch.tensor(nbr.edge_vectors(sys, dict(
                i=nl["i"][e0:e1], j=nl["j"][e0:e1], n=nl["n"][e0:e1])),
                dtype=DT, requires_grad=True)
        zs = species[a:b]
        Ei = rows_energy(hp, P, delta, zs[Il], zs[Jl], Il, zs)
        Es = Ei.sum()
        Wv = torch.zeros(3, 3, dtype=DT)
        if e1 > e0:
            (g,) = torch.autograd.grad(Es, delta, create_graph=True)
            F = torch.zeros(b - a, 3, dtype=DT).index_add(0, Il, g)
            F = F.index_add(0, Jl, -g)
            Wv = -(g[:, :, None] * delta[:, None, :]).sum(0)
        else:
            F = torch.zeros(b - a, 3, dtype=DT)
        obj = (float(grad_e_struct[s]) * Es
               + (torch.tensor(grad_forces[a:b], dtype=DT) * F).sum())
        if grad_virial is not None:
            obj = obj + (torch.tensor(grad_virial[s], dtype=DT) * Wv).sum()
        ins = [Wt] + ([pos] if want_pos else [])
        gr = torch.autograd.grad(obj, ins, allow_unused=True)
        if gr[0] is not None:
            grad = grad + gr[0]
        if want_pos and gr[1] is not None:
            gpos[a:b] = gr[1].numpy()
    out = dict(grad_weights=grad.detach().numpy())
    if want_pos:
        out["grad_pos"] = gpos
    return out


def cell_volume(cell: np.ndarray) -> float:
    """|a . (b x c)| of a cell whose rows are the lattice vectors."""
    return float(abs(np.dot(cell[0], np.cross(cell[1], cell[2]))))


def loss_and_grad(hp, weights: np.ndarray, sys, e_hat: np.ndarray,
                  f_hat: np.ndarray, nl: Optional[Dict] = None,
                  r_list: Optional[float] = None,
                  s_hat: Optional[np.ndarray] = None,
                  weights_efs=(1.0, 1.0, 1.0)) -> Dict[str, np.ndarray]:
    """L = wE mean_s((E_s - E^_s) / N_s)^2 + wF (1 / 3N) sum_i |F_i - F^_i|^2
    [+ wS (1 / 9 P) sum over the P periodic structures of |sigma_s - s^_s|^2]
    and dL/dtheta.  The paper's loss weighs per-atom energy, force and
    stress errors 8:1:1 (Model Training); the stress reading is
    sigma_s = W_s / V_s with the virial W_s = -dE/d(strain) and V_s the cell
    volume (open structures carry no stress term)."""
    hp = _as_hp(hp)
    wE, wF, wS = weights_efs
    res = energy_forces(hp, weights, sys, nl=nl, r_list=r_list)
    n_s = np.diff(sys.seg).astype(np.float64)
    B = sys.n_struct
    N = sys.n_atoms
    de = (res["e_struct"] - e_hat) / n_s
    df = res["forces"] - f_hat
    loss = float(wE * np.mean(de * de) + wF * np.sum(df * df) / (3.0 * N))
    g_e = wE * 2.0 * de / n_s / B
    g_f = wF * 2.0 * df / (3.0 * N)
    g_w = None
    sigma = None
    if s_hat is not None:
        per = np.asarray(sys.pbc, dtype=bool)
        n_p = int(per.sum())
        vol = np.array([cell_volume(sys.cell[s]) if per[s] else 1.0 for s in range(B)])
        sigma = res["virial"] / vol[:, None, None]
        ds = np.where(per[:, None, None], sigma - s_hat, 0.0)
        if n_p > 0:
            loss += float(wS * np.sum(ds * ds) / (9.0 * n_p))
            g_w = wS * 2.0 * ds / (9.0 * n_p) / vol[:, None, None]
    gw = vjp_weights(hp, weights, sys, g_e, g_f, nl=res["nl"], grad_virial=g_w)["grad_weights"]
    return dict(loss=loss, grad_weights=gw, grad_e_struct=g_e,
                grad_forces=g_f, grad_virial=g_w, e_struct=res["e_struct"],
                forces=res["forces"], stress=sigma)
