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


# ---- Nose-Hoover NVT -------------------------------------------------------

def _nh_only(K0, xi0, dt, n, Q, gkT):
    """Thermostat-only dynamics (no forces) with the oracle's splitting: a
    full step is two half steps (velocities move only by the scaling)."""
    K, xi, eta = K0, xi0, 0.0
    for _ in range(n):
        _, K, xi, eta = md.nh_half_step(K, xi, eta, dt, Q, gkT)
        _, K, xi, eta = md.nh_half_step(K, xi, eta, dt, Q, gkT)
    return K, xi, eta


def test_nh_splitting_converges_to_the_thermostat_ode():
    # dK/dt = -2 xi K, dxi/dt = (2K - gkT)/Q, deta/dt = xi, solved to 1e-13;
    # the splitting is symmetric, so its error must fall as dt^2
    from scipy.integrate import solve_ivp
    gkT, Q, K0, xi0, T = 3.0, 40.0, 2.5, 0.05, 40.0

    def f(t, y):
        K, xi, eta = y
        return [-2.0 * xi * K, (2.0 * K - gkT) / Q, xi]
    ref = solve_ivp(f, (0.0, T), [K0, xi0, 0.0], rtol=1e-13, atol=1e-15, method="DOP853").y[:, -1]
    errs = []
    for n in (100, 200, 400):
        got = np.array(_nh_only(K0, xi0, T / n, n, Q, gkT))
        errs.append(np.abs(got - ref).max())
    assert errs[-1] < 1e-4
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5


def _nvt(s=None, v0=None, **kw):
    hp, w, s0, masses, v00 = _setup()
    s = s or s0
    v0 = v00 if v0 is None else v0
    return hp, w, s, masses, v0, md.run(hp, w, s, masses, v0, 0.5, kw.pop("n", 200), skin=0.5,
                                       rebuild_every=kw.pop("rebuild", 10), **kw)


def test_nvt_conserves_the_extended_energy():
    # start at 600 K, thermostat at 300 K with a 10 fs period: the thermostat
    # moves several eV, H' = KE + PE + Q xi^2/2 + g kB T eta stays put
    hp, w, s, masses, _ = _setup()
    v0 = synth.maxwell_boltzmann(masses[s.species], 600.0, 3002)
    *_, out = _nvt(v0=v0, t_target=300.0, tau=10.0)
    h = out["log"].sum(1) + out["thermostat"][:, 2]
    drift = np.abs(h - h[0]).max() / s.n_atoms
    moved = np.abs(out["thermostat"][:, 2] - out["thermostat"][0, 2]).max() / s.n_atoms
    assert drift < 2e-3
    assert moved > 20 * drift
    # the kinetic temperature has been pulled towards the target
    m = masses[s.species]
    T = 2 * out["log"][:, 0] / (3 * s.n_atoms * synth.KB_EV)
    assert abs(T[-50:].mean() - 300.0) < abs(T[0] - 300.0)


def test_nvt_time_reversibility():
    hp, w, s, masses, v0 = _setup()
    fwd = md.run(hp, w, s, masses, v0, 0.5, 20, skin=0.5, rebuild_every=1000, t_target=300.0, tau=10.0,
                 xi0=0.01)
    xi1, eta1 = fwd["thermostat"][-1, :2]
    back = md.run(hp, w, dataclasses.replace(s, pos=fwd["pos"]), masses, -fwd["vel"], 0.5, 20, skin=0.5,
                  rebuild_every=1000, t_target=300.0, tau=10.0, xi0=-xi1, eta0=eta1)
    np.testing.assert_allclose(back["pos"], s.pos, atol=1e-9)
    np.testing.assert_allclose(-back["vel"], v0, atol=1e-10)
    np.testing.assert_allclose(-back["thermostat"][-1, 0], 0.01, atol=1e-12)
    np.testing.assert_allclose(back["thermostat"][-1, 1], 0.0, atol=1e-12)


def test_nvt_with_an_infinitely_slow_thermostat_is_nve():
    hp, w, s, masses, v0 = _setup()
    nve = md.run(hp, w, s, masses, v0, 0.5, 20, skin=0.5, rebuild_every=10)
    nvt = md.run(hp, w, s, masses, v0, 0.5, 20, skin=0.5, rebuild_every=10, t_target=300.0, tau=1e12)
    np.testing.assert_allclose(nvt["pos"], nve["pos"], atol=1e-13)
    np.testing.assert_allclose(nvt["vel"], nve["vel"], atol=1e-13)
