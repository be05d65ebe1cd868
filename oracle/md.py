"""Oracle NVE molecular dynamics (test infrastructure only).

The paper runs its production MD with a 0.5 fs time step (Methodology, MD
simulations of the C-S-H nanoparticle).  This module integrates with plain
velocity Verlet in float64, the integrator the NVE workload prescribes:

  v <- v + dt/2 * F/m * k_acc;  r <- r + dt * v;
  [every `rebuild_every` steps: wrap periodic atoms by whole lattice shifts
   and rebuild the neighbour list at r_c + skin];
  F <- F(r);  v <- v + dt/2 * F/m * k_acc,

with k_acc = 9.648533212e-3 A fs^-2 per (eV A^-1 amu^-1).  The list built at
step 0 is used for steps 1..rebuild_every-1; the rebuild happens before the
force evaluation of every step k with k % rebuild_every == 0.  Kinetic energy
KE = 1/2 sum m v^2 / k_acc (eV).  Edges in [r_c, r_c + skin) contribute zero.

Pins: time reversibility (negate v and integrate back) and bounded energy
drift on the tiny workload (tests/test_oracle_md.py).
"""

from __future__ import annotations

import dataclasses
from typing import Dict

import numpy as np

from . import model
from . import neighbors as nbr

ACC = 9.648533212e-3


def kinetic_energy(m: np.ndarray, v: np.ndarray) -> float:
    return float(0.5 * np.sum(m[:, None] * v * v) / ACC)


def run(hp, weights: np.ndarray, sys, masses_by_species: np.ndarray,
        v0: np.ndarray, dt: float, n_steps: int, skin: float,
        rebuild_every: int) -> Dict[str, np.ndarray]:
    hp = model._as_hp(hp)
    r_list = hp.r_cut + skin
    m = np.asarray(masses_by_species)[sys.species]
    pos = sys.pos.copy()
    v = v0.copy()
    cur = dataclasses.replace(sys, pos=pos)
    nl = nbr.build(cur, r_list)
    res = model.energy_forces(hp, weights, cur, nl=nl)
    F = res["forces"]
    log = [(kinetic_energy(m, v), float(res["e_struct"].sum()))]
    for k in range(1, n_steps + 1):
        v = v + 0.5 * dt * F / m[:, None] * ACC
        pos = pos + dt * v
        cur = dataclasses.replace(sys, pos=pos)
        if k % rebuild_every == 0:
            pos = nbr.wrap_positions(cur)
            cur = dataclasses.replace(sys, pos=pos)
            nl = nbr.build(cur, r_list)
        res = model.energy_forces(hp, weights, cur, nl=nl)
        F = res["forces"]
        v = v + 0.5 * dt * F / m[:, None] * ACC
        log.append((kinetic_energy(m, v), float(res["e_struct"].sum())))
    return dict(pos=pos, vel=v, forces=F, log=np.array(log))
