"""Oracle neighbour lists (test infrastructure only).

Definition followed (the paper's strictly-local cutoff neighbourhoods,
Abstract and Methodology / Model Training, radial cutoff):

  edges = {(i, j, n) : i, j in the same structure, n in Z^3 (n = 0 for an open
           structure), (i, j, n) != (i, i, 0), d^2 < r^2}
  delta = (r_j - r_i) + shift(n),  shift(n) = (n0*a + n1*b) + n2*c  (per
          component, rows a, b, c of the cell),
  d^2   = (dx*dx + dy*dy) + dz*dz,

evaluated in float64 in exactly this order with no fused multiply-add (numpy
never fuses).  The inclusion test is strict.  Canonical order is
(i, j, n0, n1, n2) ascending; rev(i, j, n) is the index of (j, i, -n).

Two independent enumerations are provided: ``brute_force`` (all pairs times
the images n = k - m_j + m_i, |k_a| <= ceil(r / w_a), with w_a the
perpendicular cell widths and m the atoms' whole-cell offsets)
and ``binned`` (a cell grid for periodic cells at least 3 bins wide).  Tests
check one against the other and against lattice-shell counts.
"""

from __future__ import annotations

import math
from typing import Dict, Optional, Sequence

import numpy as np


def perpendicular_widths(cell: np.ndarray) -> np.ndarray:
    """w_k = |det h| / |b_{k+1} x b_{k+2}| for rows b_0, b_1, b_2 of h."""
    vol = abs(float(np.linalg.det(cell)))
    w = np.empty(3)
    for k in range(3):
        cr = np.cross(cell[(k + 1) % 3], cell[(k + 2) % 3])
        w[k] = vol / math.sqrt(float(cr @ cr))
    return w


def shift_vectors(cell: np.ndarray, n: np.ndarray) -> np.ndarray:
    """shift(n) = (n0*a + n1*b) + n2*c per component, float64."""
    n = n.astype(np.float64)
    return (n[:, 0:1] * cell[0][None, :] + n[:, 1:2] * cell[1][None, :]) \
        + n[:, 2:3] * cell[2][None, :]


def _dist2(delta: np.ndarray) -> np.ndarray:
    return (delta[..., 0] * delta[..., 0] + delta[..., 1] * delta[..., 1]) \
        + delta[..., 2] * delta[..., 2]


def image_range(cell: np.ndarray, pbc: int, r: float) -> np.ndarray:
    if not pbc:
        return np.zeros(3, np.int64)
    w = perpendicular_widths(cell)
    return np.array([math.ceil(r / wk) for wk in w], np.int64)


def _images(nmax: np.ndarray) -> np.ndarray:
    rng = [np.arange(-m, m + 1) for m in nmax]
    N0, N1, N2 = np.meshgrid(*rng, indexing="ij")
    return np.stack([N0.ravel(), N1.ravel(), N2.ravel()], axis=1)  # lexicographic


def brute_force(pos: np.ndarray, cell: np.ndarray, pbc: int, r: float,
                rows: Optional[np.ndarray] = None):
    """All-pairs, all-images edge list of ONE structure.

    For periodic cells each atom's whole-cell offset m = floor(frac(r)) is
    taken out first; the images tried for the pair (i, j) are
    n = k - m_j + m_i with |k_a| <= ceil(r / w_a), which contains every n with
    |delta| < r whatever the positions.  Returns (i, j, n) arrays sorted
    canonically.  `rows` restricts the central atoms.
    """
    N = pos.shape[0]
    ks = _images(image_range(cell, pbc, r))
    if pbc:
        m = np.floor(pos @ np.linalg.inv(cell)).astype(np.int64)
    else:
        m = np.zeros((N, 3), np.int64)
    r2 = r * r
    I_out, J_out, N_out = [], [], []
    row_ids = range(N) if rows is None else rows
    jj = np.arange(N)
    for i in row_ids:
        n_all = ks[None, :, :] - m[:, None, :] + m[i][None, None, :]  # [N,K,3]
        base = pos - pos[i][None, :]                      # r_j - r_i, [N,3]
        if pbc:
            sh = shift_vectors(cell, n_all.reshape(-1, 3)).reshape(N, -1, 3)
        else:
            sh = np.zeros((N, 1, 3))
        delta = base[:, None, :] + sh                     # [N, K, 3]
        d2 = _dist2(delta)
        ok = d2 < r2
        ok[i, np.all(n_all[i] == 0, axis=1)] = False
        jjj, kk = np.nonzero(ok)                          # j-major, image-minor
        I_out.append(np.full(jjj.shape[0], i, np.int64))
        J_out.append(jj[jjj])
        N_out.append(n_all[jjj, kk] if pbc else np.zeros((jjj.shape[0], 3),
                                                         np.int64))
    if not I_out:
        return (np.zeros(0, np.int64), np.zeros(0, np.int64),
                np.zeros((0, 3), np.int64))
    return (np.concatenate(I_out), np.concatenate(J_out),
            np.concatenate(N_out, axis=0).reshape(-1, 3))


def binned(pos: np.ndarray, cell: np.ndarray, r: float,
           rows: Optional[np.ndarray] = None, chunk: int = 4096):
    """Cell-grid edge list of ONE periodic structure whose perpendicular widths
    hold at least 3 bins of width > r.  Positions need not be wrapped: each
    atom's image offset m = floor(frac) is folded into n.  Same output as
    `brute_force`.
    """
    w = perpendicular_widths(cell)
    nb = np.array([int(math.floor(wk / (r * (1.0 + 1e-9)))) for wk in w])
    if np.any(nb < 3):
        raise ValueError("cell too small for binning; use brute_force")
    inv = np.linalg.inv(cell)
    frac = pos @ inv
    m = np.floor(frac).astype(np.int64)
    fw = frac - m
    b = np.minimum(np.floor(fw * nb[None, :]).astype(np.int64), nb[None, :] - 1)
    flat = (b[:, 0] * nb[1] + b[:, 1]) * nb[2] + b[:, 2]
    order = np.argsort(flat, kind="stable")
    counts = np.bincount(flat, minlength=int(np.prod(nb)))
    start = np.zeros(counts.shape[0] + 1, np.int64)
    start[1:] = np.cumsum(counts)
    r2 = r * r
    offs = _images(np.array([1, 1, 1]))
    row_ids = np.arange(pos.shape[0]) if rows is None else np.asarray(rows)
    I_out, J_out, N_out = [], [], []
    for c0 in range(0, row_ids.shape[0], chunk):
        ids = row_ids[c0:c0 + chunk]
        cand_i, cand_j, cand_n = [], [], []
        for o in offs:
            nbp = b[ids] + o[None, :]
            wrap = np.floor_divide(nbp, nb[None, :])
            nbw = nbp - wrap * nb[None, :]
            cf = (nbw[:, 0] * nb[1] + nbw[:, 1]) * nb[2] + nbw[:, 2]
            cnt = counts[cf]
            tot = int(cnt.sum())
            if tot == 0:
                continue
            rep_i = np.repeat(ids, cnt)
            rep_wrap = np.repeat(wrap, cnt, axis=0)
            st = np.repeat(start[cf], cnt)
            within = np.arange(tot) - np.repeat(np.cumsum(cnt) - cnt, cnt)
            jj = order[st + within]
            # delta = w_j - w_i + wrap*h = r_j - r_i + (wrap - m_j + m_i) h
            n = rep_wrap - m[jj] + m[rep_i]
            cand_i.append(rep_i)
            cand_j.append(jj)
            cand_n.append(n)
        ci = np.concatenate(cand_i)
        cj = np.concatenate(cand_j)
        cn = np.concatenate(cand_n, axis=0)
        delta = (pos[cj] - pos[ci]) + shift_vectors(cell, cn)
        d2 = _dist2(delta)
        ok = (d2 < r2) & ~((ci == cj) & np.all(cn == 0, axis=1))
        I_out.append(ci[ok])
        J_out.append(cj[ok])
        N_out.append(cn[ok])
    I = np.concatenate(I_out)
    J = np.concatenate(J_out)
    Nn = np.concatenate(N_out, axis=0)
    key = np.lexsort((Nn[:, 2], Nn[:, 1], Nn[:, 0], J, I))
    return I[key], J[key], Nn[key]


def build(sys, r: float, rows: Optional[np.ndarray] = None,
          method: str = "auto") -> Dict[str, np.ndarray]:
    """Canonical CSR edge list of a whole batch (global atom indices).

    Returns dict with i, j (int64), n (int64 [E,3]), row_ptr ([N+1]) and rev
    (index of the reverse edge; -1 where `rows` left it out).
    """
    Is, Js, Ns = [], [], []
    for s in range(sys.n_struct):
        a, b = int(sys.seg[s]), int(sys.seg[s + 1])
        pos = sys.pos[a:b]
        cell = sys.cell[s]
        pbc = int(sys.pbc[s])
        sub_rows = None
        if rows is not None:
            sel = rows[(rows >= a) & (rows < b)] - a
            if sel.shape[0] == 0:
                continue
            sub_rows = sel
        use_bins = False
        if method in ("auto", "binned") and pbc:
            w = perpendicular_widths(cell)
            use_bins = bool(np.all(np.floor(w / (r * (1.0 + 1e-9))) >= 3))
            if method == "binned" and not use_bins:
                raise ValueError("binned method needs >= 3 bins per axis")
        if use_bins and (method == "binned" or (b - a) > 2000):
            i, j, n = binned(pos, cell, r, rows=sub_rows)
        else:
            i, j, n = brute_force(pos, cell, pbc, r, rows=sub_rows)
        Is.append(i + a)
        Js.append(j + a)
        Ns.append(n)
    if Is:
        I = np.concatenate(Is)
        J = np.concatenate(Js)
        Nn = np.concatenate(Ns, axis=0)
    else:
        I = np.zeros(0, np.int64)
        J = np.zeros(0, np.int64)
        Nn = np.zeros((0, 3), np.int64)
    row_ptr = np.zeros(sys.n_atoms + 1, np.int64)
    np.add.at(row_ptr, I + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    rev = reverse_index(I, J, Nn)
    return dict(i=I, j=J, n=Nn, row_ptr=row_ptr, rev=rev)


def reverse_index(I: np.ndarray, J: np.ndarray, Nn: np.ndarray) -> np.ndarray:
    """rev[e] = index of (j, i, -n), found by a dictionary lookup; -1 if the
    reverse edge is not in the list."""
    look = {}
    for e in range(I.shape[0]):
        look[(int(I[e]), int(J[e]), int(Nn[e, 0]), int(Nn[e, 1]),
              int(Nn[e, 2]))] = e
    rev = np.full(I.shape[0], -1, np.int64)
    for e in range(I.shape[0]):
        rev[e] = look.get((int(J[e]), int(I[e]), -int(Nn[e, 0]),
                           -int(Nn[e, 1]), -int(Nn[e, 2])), -1)
    return rev


def edge_vectors(sys, nl: Dict[str, np.ndarray]) -> np.ndarray:
    """delta_e = (r_j - r_i) + shift(n) in float64, in the canonical order."""
    E = nl["i"].shape[0]
    if E == 0:
        return np.zeros((0, 3))
    struct = np.searchsorted(sys.seg, nl["i"], side="right") - 1
    out = np.empty((E, 3))
    for s in np.unique(struct):
        sel = struct == s
        base = sys.pos[nl["j"][sel]] - sys.pos[nl["i"][sel]]
        if sys.pbc[s]:
            out[sel] = base + shift_vectors(sys.cell[s], nl["n"][sel])
        else:
            out[sel] = base + np.zeros((1, 3))
    return out


def wrap_positions(sys):
    """Return positions with each periodic atom moved into the cell by a whole
    lattice shift: r' = r - shift(floor(frac(r))).  Atoms already inside are
    left bit-identical."""
    pos = sys.pos.copy()
    for s in range(sys.n_struct):
        if not sys.pbc[s]:
            continue
        a, b = int(sys.seg[s]), int(sys.seg[s + 1])
        frac = pos[a:b] @ np.linalg.inv(sys.cell[s])
        n = np.floor(frac).astype(np.int64)
        move = np.any(n != 0, axis=1)
        if np.any(move):
            pos[a:b][move] = pos[a:b][move] - shift_vectors(sys.cell[s], n[move])
    return pos
