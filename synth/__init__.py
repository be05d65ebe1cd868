"""Seeded synthetic inputs shared by the FP64 oracle and the HIP path.

This module holds none of the method's arithmetic: it draws structures
(positions, species, cells, periodicity flags, segment offsets), masses,
initial velocities, training targets and raw weight values from fixed seeds.
Both sides consume exactly these arrays.  The weight *layout* (which block has
which fan-in) is supplied by the caller, so the model structure lives on each
side independently.

Workload recipes (the paper's own workloads -- the T11 crystal, the C-S-H
nanoparticle, the MPtrj/OFF23/Transition1x sets -- are not available, so
these seeded systems stand in for them):

* ``A``  32 of the 64 sites of a 4x4x4 simple-cubic lattice (a = 2.0 A,
  periodic 8 A cube), uniform +-0.3 A jitter, 16 + 16 atoms of 2 species.
* ``B``  24^3 simple-cubic lattice, a = 2.2 A, +-0.25 A jitter, 4 species drawn
  uniformly, periodic 52.8 A cube (13,824 atoms).
* ``C``  64 open clusters, N ~ U{20..200}, 10 species, uniform in a sphere of
  density 0.1 A^-3 with 0.9 A rejection.
* ``D``  512 structures, N log-uniform in [8, 300], half periodic random
  triclinic cells, half open clusters, density U(0.08, 0.12) A^-3, 89 species.
* ``E``  100^3 simple-cubic lattice, a = 2.3 A, +-0.25 A jitter, 4 species,
  per-species masses U(1, 60) amu, Maxwell-Boltzmann velocities at 300 K.

Every generator uses ``numpy.random.Generator(PCG64(seed))`` and documents its
draw order so that results are reproducible bit for bit.
"""

from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence

import numpy as np

# Unit conventions: positions in Angstrom, energies in eV, masses in amu,
# time in fs.  1 eV / (amu * A^2 / fs^2) conversion used for velocities.
ACC_UNIT = 9.648533212e-3          # (eV / A / amu) -> A / fs^2
KB_EV = 8.617333262e-5             # Boltzmann constant, eV / K

STRUCT_SEEDS = {"A": 1001, "B": 1002, "C": 1003, "D": 1004, "E": 1005}
WEIGHT_SEEDS = {"A": 2001, "B": 2002, "C": 2003, "D": 2004, "E": 2005}
VELOCITY_SEED_E = 3005
TARGET_SEED_C = 4003


@dataclasses.dataclass
class System:
    """A batch of structures flattened by segment offsets.

    pos      [N, 3] float64, Angstrom (used as given, never wrapped here)
    species  [N]    int32 in [0, n_species)
    cell     [B, 3, 3] float64, rows are the lattice vectors a, b, c
    pbc      [B]    uint8, 1 = periodic in all three directions, 0 = open
    seg      [B+1]  int64 atom offsets of each structure
    """

    pos: np.ndarray
    species: np.ndarray
    cell: np.ndarray
    pbc: np.ndarray
    seg: np.ndarray
    n_species: int

    @property
    def n_atoms(self) -> int:
        return int(self.pos.shape[0])

    @property
    def n_struct(self) -> int:
        return int(self.cell.shape[0])

    def structure(self, s: int) -> "System":
        a, b = int(self.seg[s]), int(self.seg[s + 1])
        return System(self.pos[a:b].copy(), self.species[a:b].copy(),
                      self.cell[s:s + 1].copy(), self.pbc[s:s + 1].copy(),
                      np.array([0, b - a], dtype=np.int64), self.n_species)


def _pack(parts: Sequence[System], n_species: int) -> System:
    pos = np.concatenate([p.pos for p in parts], axis=0)
    species = np.concatenate([p.species for p in parts]).astype(np.int32)
    cell = np.concatenate([p.cell for p in parts], axis=0)
    pbc = np.concatenate([p.pbc for p in parts]).astype(np.uint8)
    sizes = [p.n_atoms for p in parts]
    seg = np.zeros(len(parts) + 1, dtype=np.int64)
    seg[1:] = np.cumsum(sizes)
    return System(pos, species, cell, pbc, seg, n_species)


def cubic_lattice(n_side: int, spacing: float, jitter: float, n_species: int,
                  seed: int) -> System:
    """Jittered simple-cubic lattice in a periodic cube of side n_side*spacing.

    Draw order: jitter U(-jitter, jitter) of shape [N, 3], then species
    integers U{0..n_species-1} of shape [N].
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    g = np.arange(n_side, dtype=np.float64) * spacing
    # site order: x slowest, z fastest
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    sites = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    n = sites.shape[0]
    pos = sites + rng.uniform(-jitter, jitter, size=(n, 3))
    species = rng.integers(0, n_species, size=n).astype(np.int32)
    L = n_side * spacing
    cell = (np.eye(3) * L)[None]
    return System(pos, species, cell, np.ones(1, np.uint8),
                  np.array([0, n], np.int64), n_species)


def config_a() -> System:
    """32 of the 64 sites of a 4x4x4 lattice (a = 2.0 A) in an 8 A cube.

    Draw order: permutation of the 64 sites (first 32 kept, in ascending site
    order), jitter U(-0.3, 0.3) [32, 3], permutation of 32 for species
    (first 16 -> species 0, rest -> species 1).
    """
    rng = np.random.Generator(np.random.PCG64(STRUCT_SEEDS["A"]))
    g = np.arange(4, dtype=np.float64) * 2.0
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    sites = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    keep = np.sort(rng.permutation(64)[:32])
    pos = sites[keep] + rng.uniform(-0.3, 0.3, size=(32, 3))
    perm = rng.permutation(32)
    species = np.zeros(32, np.int32)
    species[perm[16:]] = 1
    cell = (np.eye(3) * 8.0)[None]
    return System(pos, species, cell, np.ones(1, np.uint8),
                  np.array([0, 32], np.int64), 2)


def config_b() -> System:
    return cubic_lattice(24, 2.2, 0.25, 4, STRUCT_SEEDS["B"])


def _cluster(rng: np.random.Generator, n: int, density: float, dmin: float,
             n_species: int) -> System:
    """Uniform points in a sphere of radius (3n/(4 pi rho))^(1/3), each new
    point rejected if closer than dmin to an accepted one.  Draw order per
    attempt: 3 uniforms in the bounding cube [-R, R]^3 (points outside the
    sphere are rejected too); after placement, species integers [n]."""
    R = (3.0 * n / (4.0 * math.pi * density)) ** (1.0 / 3.0)
    pts = np.empty((n, 3))
    k = 0
    d2min = dmin * dmin
    while k < n:
        p = rng.uniform(-R, R, size=3)
        if p @ p >= R * R:
            continue
        if k > 0:
            dd = pts[:k] - p
            if np.min(np.einsum("ij,ij->i", dd, dd)) < d2min:
                continue
        pts[k] = p
        k += 1
    species = rng.integers(0, n_species, size=n).astype(np.int32)
    return System(pts, species, np.zeros((1, 3, 3)), np.zeros(1, np.uint8),
                  np.array([0, n], np.int64), n_species)


def _triclinic(rng: np.random.Generator, n: int, density: float, dmin: float,
               n_species: int) -> System:
    """Random triclinic periodic cell h = I + U(-0.2, 0.2)^{3x3} rescaled so
    that det h = n / density; fractional coordinates uniform with a 0.9 A
    rejection against the 27 nearest images of every accepted atom.  Draw
    order: the 9 cell perturbations, then 3 uniforms per attempt, then
    species [n]."""
    h = np.eye(3) + rng.uniform(-0.2, 0.2, size=(3, 3))
    det = np.linalg.det(h)
    if det < 0:
        h[2] = -h[2]
        det = -det
    h = h * (n / density / det) ** (1.0 / 3.0)
    imgs = np.array([[i, j, k] for i in (-1, 0, 1) for j in (-1, 0, 1)
                     for k in (-1, 0, 1)], dtype=np.float64) @ h
    pts = np.empty((n, 3))
    k = 0
    d2min = dmin * dmin
    while k < n:
        f = rng.uniform(0.0, 1.0, size=3)
        p = f @ h
        if k > 0:
            dd = (pts[:k, None, :] - p[None, None, :]) + imgs[None, :, :]
            if np.min(np.einsum("abi,abi->ab", dd, dd)) < d2min:
                continue
        pts[k] = p
        k += 1
    species = rng.integers(0, n_species, size=n).astype(np.int32)
    return System(pts, species, h[None].copy(), np.ones(1, np.uint8),
                  np.array([0, n], np.int64), n_species)


def clusters(n_struct: int, n_lo: int, n_hi: int, density: float, dmin: float,
             n_species: int, seed: int) -> System:
    """Batch of open clusters with N ~ U{n_lo..n_hi} (draw: all sizes first)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = rng.integers(n_lo, n_hi + 1, size=n_struct)
    parts = [_cluster(rng, int(n), density, dmin, n_species) for n in sizes]
    return _pack(parts, n_species)


def config_c() -> System:
    return clusters(64, 20, 200, 0.1, 0.9, 10, STRUCT_SEEDS["C"])


def config_d(n_struct: int = 512) -> System:
    """Uneven batch: sizes log-uniform in [8, 300] (rounded), densities
    U(0.08, 0.12), even-indexed structures periodic triclinic, odd-indexed
    open clusters.  Draw order: sizes [n_struct], densities [n_struct], then
    each structure in turn."""
    rng = np.random.Generator(np.random.PCG64(STRUCT_SEEDS["D"]))
    sizes = np.rint(np.exp(rng.uniform(math.log(8.0), math.log(300.0),
                                       size=n_struct))).astype(np.int64)
    dens = rng.uniform(0.08, 0.12, size=n_struct)
    parts = []
    for s in range(n_struct):
        if s % 2 == 0:
            parts.append(_triclinic(rng, int(sizes[s]), float(dens[s]), 0.9, 89))
        else:
            parts.append(_cluster(rng, int(sizes[s]), float(dens[s]), 0.9, 89))
    return _pack(parts, 89)


def mixed_batch(n_struct: int, n_lo: int, n_hi: int, density: float, n_species: int,
                seed: int) -> System:
    """Small stand-in for a training batch with stress: even-indexed
    structures periodic triclinic, odd-indexed open clusters, N ~ U{n_lo..n_hi}
    (draw: all sizes first, then each structure in turn), d_min 0.9 A."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = rng.integers(n_lo, n_hi + 1, size=n_struct)
    parts = []
    for s in range(n_struct):
        if s % 2 == 0:
            parts.append(_triclinic(rng, int(sizes[s]), density, 0.9, n_species))
        else:
            parts.append(_cluster(rng, int(sizes[s]), density, 0.9, n_species))
    return _pack(parts, n_species)


def stress_targets(sys: System, seed: int, scale: float = 0.01) -> np.ndarray:
    """Target stresses N(0, scale^2) eV/A^3 per component for the periodic
    structures, zeros for the open ones ([n_struct, 3, 3])."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = scale * rng.standard_normal(size=(sys.n_struct, 3, 3))
    return np.where(np.asarray(sys.pbc, dtype=bool)[:, None, None], t, 0.0)


def config_e(n_side: int = 100) -> System:
    return cubic_lattice(n_side, 2.3, 0.25, 4, STRUCT_SEEDS["E"])


def species_masses(n_species: int, seed: int, lo: float = 1.0,
                   hi: float = 60.0) -> np.ndarray:
    """One mass per species, U(lo, hi) amu."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(lo, hi, size=n_species)


def maxwell_boltzmann(masses_per_atom: np.ndarray, temperature: float,
                      seed: int) -> np.ndarray:
    """Velocities in A/fs: v ~ N(0, kT/m) per component, centre-of-mass
    velocity removed, then rescaled so that the kinetic temperature with
    3N - 3 degrees of freedom is exactly `temperature`."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m = np.asarray(masses_per_atom, dtype=np.float64)
    n = m.shape[0]
    std = np.sqrt(KB_EV * temperature * ACC_UNIT / m)
    v = rng.standard_normal(size=(n, 3)) * std[:, None]
    v -= (m[:, None] * v).sum(0) / m.sum()
    ke = 0.5 * np.sum(m[:, None] * v * v) / ACC_UNIT
    t_now = 2.0 * ke / ((3 * n - 3) * KB_EV)
    return v * math.sqrt(temperature / t_now)


def training_targets(sys: System, seed: int = TARGET_SEED_C):
    """E_hat_s = N_s * N(0,1) eV, F_hat ~ N(0,1) eV/A (draw order: E then F)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n_s = np.diff(sys.seg).astype(np.float64)
    e_hat = n_s * rng.standard_normal(size=sys.n_struct)
    f_hat = rng.standard_normal(size=(sys.n_atoms, 3))
    return e_hat, f_hat


def draw_weights(blocks: Sequence[Dict], seed: int) -> np.ndarray:
    """Flat float64 weight vector from a block table.

    Each block is a dict with ``size`` and ``init``:
      * ``"fan_in"``: N(0, 1/fan_in) with the block's ``fan_in``;
      * ``"normal"``: N(0, 1);
      * ``"ones"``:   all ones (no draw).
    Blocks are filled in table order from one PCG64 stream.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for b in blocks:
        size = int(b["size"])
        kind = b["init"]
        if kind == "fan_in":
            out.append(rng.standard_normal(size) / math.sqrt(float(b["fan_in"])))
        elif kind == "normal":
            out.append(rng.standard_normal(size))
        elif kind == "ones":
            out.append(np.ones(size))
        else:
            raise ValueError(f"unknown init kind {kind!r}")
    return np.concatenate(out) if out else np.zeros(0)


def perturb_positions(sys: System, scale: float, seed: int) -> System:
    """Copy of `sys` with positions displaced by U(-scale, scale)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return dataclasses.replace(sys, pos=sys.pos + rng.uniform(-scale, scale,
                                                              size=sys.pos.shape))


# ---------------------------------------------------------------------------
# Hyperparameters of the five workloads.  Plain data; the derived numbers
# avg_num_neighbors and energy_scale are frozen values measured by the oracle
# and stored in tests/golden/hparams.json (see load_hparams).

CONFIGS: Dict[str, Dict] = {
    "A": dict(n_species=2, l_max=1, n_layers=1, latent=32, channels=8,
              n_bessel=8, poly_p=6, twobody=[16, 32], latent_depth=2,
              edge_hidden=32, r_cut=4.0, r_list=4.0),
    "B": dict(n_species=4, l_max=2, n_layers=2, latent=256, channels=64,
              n_bessel=8, poly_p=6, twobody=[64, 128, 256], latent_depth=3,
              edge_hidden=128, r_cut=5.5, r_list=5.5),
    "C": dict(n_species=10, l_max=2, n_layers=2, latent=128, channels=32,
              n_bessel=8, poly_p=6, twobody=[32, 64, 128], latent_depth=3,
              edge_hidden=128, r_cut=5.0, r_list=5.0),
    "D": dict(n_species=89, l_max=2, n_layers=3, latent=256, channels=64,
              n_bessel=8, poly_p=6, twobody=[64, 128, 256], latent_depth=3,
              edge_hidden=128, r_cut=6.0, r_list=6.0),
    "E": dict(n_species=4, l_max=2, n_layers=3, latent=256, channels=64,
              n_bessel=8, poly_p=6, twobody=[64, 128, 256], latent_depth=3,
              edge_hidden=128, r_cut=5.5, r_list=6.0),
}

SYSTEMS = {"A": config_a, "B": config_b, "C": config_c, "D": config_d,
           "E": config_e}


def load_hparams(name: str, golden_path: Optional[str] = None) -> Dict:
    """Config dict with the frozen avg_num_neighbors and energy_scale."""
    import json
    import os
    hp = dict(CONFIGS[name])
    if golden_path is None:
        golden_path = os.path.join(os.path.dirname(os.path.dirname(
            os.path.abspath(__file__))), "tests", "golden", "hparams.json")
    with open(golden_path) as f:
        frozen = json.load(f)
    hp.update(frozen[name]["frozen"])
    return hp


def subset_rows(n_atoms: int, k: int, seed: int) -> np.ndarray:
    """k distinct atom indices, sorted, from a seeded permutation."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.sort(rng.permutation(n_atoms)[:k]).astype(np.int64)
