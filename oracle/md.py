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

Canonical (NVT) runs: the paper thermalises its systems at 300 K in the NVT
ensemble (Results, Fig. 2; the C-S-H nanoparticle run) without naming the
thermostat.  The reading taken here is a single Nose-Hoover thermostat
(friction xi, position eta, mass Q = g kB T tau^2 for g degrees of freedom
and period tau) integrated by the symmetric Trotter splitting of Martyna,
Tuckerman and Klein: a thermostat half step of dt/2, the velocity Verlet
step, a second thermostat half step.  A thermostat half step advances xi by
dt/4 with G = (2 KE - g kB T) / Q, scales every velocity by
exp(-xi dt / 2), advances eta by xi dt / 2, and advances xi by dt/4 again
with G of the scaled velocities.  H' = KE + PE + Q xi^2 / 2 + g kB T eta is
conserved by the exact dynamics.

Pins (NVT): the thermostat-only dynamics (no forces) against a fine ODE
solution, conservation of H', time reversibility with (v, xi) negated, and
the tau -> infinity limit, which is the NVE integrator.
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


KB_EV = 8.617333262e-5   # eV / K


def nh_half_step(ke: float, xi: float, eta: float, dt: float, Q: float, gkT: float):
    """One thermostat half step (time dt/2) of the Nose-Hoover splitting:
    returns (velocity scale, KE after scaling, xi, eta)."""
    xi = xi + 0.25 * dt * (2.0 * ke - gkT) / Q
    scale = float(np.exp(-0.5 * dt * xi))
    ke = ke * scale * scale
    eta = eta + 0.5 * dt * xi
    xi = xi + 0.25 * dt * (2.0 * ke - gkT) / Q
    return scale, ke, xi, eta


def run(hp, weights: np.ndarray, sys, masses_by_species: np.ndarray,
        v0: np.ndarray, dt: float, n_steps: int, skin: float,
        rebuild_every: int, t_target: float = 0.0, tau: float = 0.0,
        n_dof: int = 0, xi0: float = 0.0, eta0: float = 0.0) -> Dict[str, np.ndarray]:
    """NVE (t_target <= 0) or Nose-Hoover NVT trajectory.  log rows are
    (KE, PE) after each step (row 0: the start); thermostat rows are
    (xi, eta, Q xi^2/2 + g kB T eta)."""
    hp = model._as_hp(hp)
    r_list = hp.r_cut + skin
    m = np.asarray(masses_by_species)[sys.species]
    pos = sys.pos.copy()
    v = v0.copy()
    nvt = t_target > 0.0
    g = n_dof if n_dof > 0 else 3 * sys.n_atoms
    gkT = g * KB_EV * t_target
    Q = gkT * tau * tau if nvt else 1.0
    xi, eta = float(xi0), float(eta0)
    cur = dataclasses.replace(sys, pos=pos)
    nl = nbr.build(cur, r_list)
    res = model.energy_forces(hp, weights, cur, nl=nl)
    F = res["forces"]
    log = [(kinetic_energy(m, v), float(res["e_struct"].sum()))]
    thermo = [(xi, eta, 0.5 * Q * xi * xi + gkT * eta)]
    for k in range(1, n_steps + 1):
        if nvt:
            sc, _, xi, eta = nh_half_step(kinetic_energy(m, v), xi, eta, dt, Q, gkT)
            v = v * sc
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
        if nvt:
            sc, _, xi, eta = nh_half_step(kinetic_energy(m, v), xi, eta, dt, Q, gkT)
            v = v * sc
        log.append((kinetic_energy(m, v), float(res["e_struct"].sum())))
        thermo.append((xi, eta, 0.5 * Q * xi * xi + gkT * eta))
    return dict(pos=pos, vel=v, forces=F, log=np.array(log), thermostat=np.array(thermo))
