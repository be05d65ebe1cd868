"""Pins of the oracle integrator: time reversibility and bounded NVE drift on
the tiny periodic workload; Maxwell-Boltzmann initial temperature."""

import dataclasses

import numpy as np

import synth
from oracle import md
from oracle import model as M


def _setup():
    hp = synth.load_hparams("A")
    hpo = M.HParams.from_dict(hp)
    w = synth.draw_weights(M.param_layout(hpo), synth.WEIGHT_SEEDS["A"])
    s = synth.config_a()
    masses = np.array([12.0, 16.0])
    v0 = synth.maxwell_boltzmann(masses[s.species], 300.0, 3001)
    return hpo, w, s, masses, v0


def test_initial_temperature_and_momentum():
    _, _, s, masses, v0 = _setup()
    m = masses[s.species]
    np.testing.assert_allclose((m[:, None] * v0).sum(0), 0, atol=1e-14)
    ke = md.kinetic_energy(m, v0)
    T = 2 * ke / ((3 * s.n_atoms - 3) * synth.KB_EV)
    assert abs(T - 300.0) < 1e-9


def test_time_reversibility_fixed_list():
    hp, w, s, masses, v0 = _setup()
    fwd = md.run(hp, w, s, masses, v0, 0.5, 20, skin=0.5, rebuild_every=1000)
    back = md.run(hp, w, dataclasses.replace(s, pos=fwd["pos"]), masses,
                  -fwd["vel"], 0.5, 20, skin=0.5, rebuild_every=1000)
    np.testing.assert_allclose(back["pos"], s.pos, atol=1e-9)
    np.testing.assert_allclose(-back["vel"], v0, atol=1e-10)


def test_nve_drift_small():
    hp, w, s, masses, v0 = _setup()
    out = md.run(hp, w, s, masses, v0, 0.5, 200, skin=0.5, rebuild_every=10)
    etot = out["log"].sum(1)
    drift = np.abs(etot - etot[0]).max() / s.n_atoms
    ke_scale = out["log"][:, 0].std() / s.n_atoms
    assert drift < 2e-3          # eV/atom over 100 fs with dt = 0.5 fs
    assert drift < 0.1 * max(ke_scale, 1e-3) or drift < 5e-4
