"""GPU MD step: trajectory parity with the FP64 oracle integrator (FP32
forces), bitwise equality of graph replays and eager steps, the skin flag,
and NVE / NVT drift with BF16 forces bounded by the same trajectory's drift
with FP32 forces."""

import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

# BF16 energy gate against FP64, eV/atom
BF16_E_GATE = 1e-3


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _setup(precision, s=None, cfg="A", use_graph=False, skin=0.5, rebuild=10, v0=None, **nvt):
    import paper_2502_06073_amd as afm
    from oracle import model as M
    hp = synth.load_hparams(cfg)
    s = s or synth.SYSTEMS[cfg]()
    w = synth.draw_weights(M.param_layout(M.HParams.from_dict(hp)), synth.WEIGHT_SEEDS[cfg])
    masses = synth.species_masses(hp["n_species"], 3005)
    if v0 is None:
        v0 = synth.maxwell_boltzmann(masses[s.species], 300.0, 3001)
    model = afm.Model(hp, w, precision=precision)
    sysd = afm.DeviceSystem.from_synth(s)
    calc = afm.Calculator(model, sysd, r_list=hp["r_cut"] + skin)
    md = afm.MD(calc, masses, v0, dt_fs=0.5, skin=skin, rebuild_every=rebuild, use_graph=use_graph, **nvt)
    return hp, w, s, masses, v0, md


def test_md_matches_oracle_fp32():
    import torch
    from oracle import md as omd
    hp, w, s, masses, v0, md = _setup("fp32")
    log = md.run(20).cpu().numpy()
    torch.cuda.synchronize()
    pos = md.calc.sysd.pos.cpu().numpy()
    vel = md.vel.cpu().numpy()
    ref = omd.run(hp, w, s, masses, v0, 0.5, 20, skin=0.5, rebuild_every=10)
    dpos = np.abs(pos - ref["pos"]).max()
    dvel = np.abs(vel - ref["vel"]).max()
    de = np.abs(log - ref["log"][1:]).max()
    _say(f"[md fp32] max|dr| {dpos:.2e} A, max|dv| {dvel:.2e}, max|dE| {de:.2e} eV")
    assert dpos < 1e-5 and dvel < 1e-5
    assert de < 1e-4 * s.n_atoms
    assert md.calc.status() == 0


def test_md_graph_replay_equals_eager():
    import torch
    _, _, _, _, _, eager = _setup("fp32", use_graph=False)
    _, _, _, _, _, graph = _setup("fp32", use_graph=True)
    logs_e, logs_g = [], []
    for rep in range(4):            # step 0 eager, then capture, then replays
        logs_e.append(eager.run(10).cpu().numpy())
        logs_g.append(graph.run(10).cpu().numpy())
        torch.cuda.synchronize()
        _ = eager.calc.sysd.pos.sum().item()   # eager work between replays
        np.testing.assert_array_equal(logs_e[-1], logs_g[-1])
        np.testing.assert_array_equal(eager.calc.sysd.pos.cpu().numpy(), graph.calc.sysd.pos.cpu().numpy())
        np.testing.assert_array_equal(eager.vel.cpu().numpy(), graph.vel.cpu().numpy())
    _say("[md graph] 4 x 10 steps bitwise equal")


def test_md_skin_flag_forced_from_host():
    # skin 0: any displacement exceeds skin/2, the flag must be raised
    _, _, _, _, _, md = _setup("fp32", skin=0.0, rebuild=1000)
    md.run(2)
    assert md.calc.status() & 8


def test_md_bf16_energy_drift_small():
    s = synth.cubic_lattice(6, 2.3, 0.25, 4, 99)
    # the random-weight lattice heats up to ~1700 K; light atoms then move
    # up to ~0.07 A/fs, so the list is rebuilt every 2 fs to stay within the
    # half-skin bound
    # The same trajectory with FP32 forces sets the bound: velocity Verlet's
    # own O(dt^2) energy fluctuation at this temperature is the floor, and
    # the BF16 forces may add at most a few times that.  The BF16 potential
    # energy is itself evaluated with an error (bf16 activations, up to the
    # 1 meV/atom energy gate), which changes with the configuration: the
    # logged E(t) - E(0) can carry that error twice, at t and at 0.
    drifts = {}
    for prec in ("fp32", "bf16"):
        hp, w, s, masses, v0, md = _setup(prec, s=s, cfg="E", rebuild=4)
        log = md.run(100).cpu().numpy()
        e = log.sum(1)
        drifts[prec] = np.abs(e - e[0]).max() / s.n_atoms
        _say(f"[md {prec}] 100 steps: max |E(t)-E(0)|/N = {drifts[prec] * 1e3:.4f} meV/atom; "
             f"KE/N {log[:, 0].mean() / s.n_atoms:.3f}")
        assert md.calc.status() == 0
    assert drifts["bf16"] <= 5.0 * drifts["fp32"] + 2 * BF16_E_GATE


def test_md_cutoff_compaction_matches_full_list():
    """With a skin, the MD step evaluates forces on the list restricted to
    |delta| < r_cut; at the same positions the full r_cut + skin list must
    give the same forces and energies (skin edges contribute exactly zero),
    up to the summation order of the environment sums."""
    import torch
    s = synth.cubic_lattice(6, 2.3, 0.25, 4, 98)
    hp, w, s, masses, v0, md = _setup("fp32", s=s, cfg="E", rebuild=3)
    md.run(5)
    torch.cuda.synchronize()
    F_md = md.forces.cpu().numpy().copy()
    E_md = md.e_atom.cpu().numpy().copy()
    nl_listed = int(md.calc.nl.n_edges.item())
    md.calc.build_neighbors()
    out = md.calc.energy_forces(virial=False)
    F = out["forces"].cpu().numpy()
    E = out["e_atom"].cpu().numpy()
    rel_f = np.linalg.norm(F_md - F) / np.linalg.norm(F)
    rel_e = np.linalg.norm(E_md - E) / np.linalg.norm(E)
    _say(f"[md compaction] listed edges {nl_listed}; force rel {rel_f:.2e}, e_atom rel {rel_e:.2e}")
    assert rel_f < 1e-5 and rel_e < 1e-5
    assert md.calc.status() == 0


# ---- Nose-Hoover NVT -------------------------------------------------------

def _hot_v0(cfg="A", s=None):
    hp = synth.load_hparams(cfg)
    s = s or synth.SYSTEMS[cfg]()
    masses = synth.species_masses(hp["n_species"], 3005)
    return synth.maxwell_boltzmann(masses[s.species], 600.0, 3002)


def test_md_nvt_matches_oracle_fp32():
    import torch
    from oracle import md as omd
    v0 = _hot_v0()
    hp, w, s, masses, v0, md = _setup("fp32", v0=v0, t_target_K=300.0, tau_fs=10.0)
    log = md.run(20).cpu().numpy()
    torch.cuda.synchronize()
    tlog = md.thermostat_log.cpu().numpy()
    nh = md.nh.cpu().numpy()
    ref = omd.run(hp, w, s, masses, v0, 0.5, 20, skin=0.5, rebuild_every=10, t_target=300.0, tau=10.0)
    dpos = np.abs(md.calc.sysd.pos.cpu().numpy() - ref["pos"]).max()
    dvel = np.abs(md.vel.cpu().numpy() - ref["vel"]).max()
    de = np.abs(log - ref["log"][1:]).max()
    dth = np.abs(tlog - ref["thermostat"][1:, 2]).max()
    _say(f"[md nvt fp32] max|dr| {dpos:.2e} A, max|dv| {dvel:.2e}, max|dE| {de:.2e} eV, "
         f"max|d thermostat| {dth:.2e} eV; xi {nh[0]:.4e} (oracle {ref['thermostat'][-1, 0]:.4e})")
    assert dpos < 1e-5 and dvel < 1e-5
    assert de < 1e-4 * s.n_atoms and dth < 1e-4 * s.n_atoms
    np.testing.assert_allclose(nh[:2], ref["thermostat"][-1, :2], rtol=1e-4, atol=1e-9)
    assert md.calc.status() == 0


def test_md_nvt_graph_replay_equals_eager():
    import torch
    v0 = _hot_v0()
    _, _, _, _, _, eager = _setup("fp32", v0=v0, t_target_K=300.0, tau_fs=10.0)
    _, _, _, _, _, graph = _setup("fp32", v0=v0, use_graph=True, t_target_K=300.0, tau_fs=10.0)
    for rep in range(4):
        le = eager.run(10).cpu().numpy()
        lg = graph.run(10).cpu().numpy()
        torch.cuda.synchronize()
        _ = eager.calc.sysd.pos.sum().item()
        np.testing.assert_array_equal(le, lg)
        np.testing.assert_array_equal(eager.thermostat_log.cpu().numpy(), graph.thermostat_log.cpu().numpy())
        np.testing.assert_array_equal(eager.nh.cpu().numpy(), graph.nh.cpu().numpy())
        np.testing.assert_array_equal(eager.vel.cpu().numpy(), graph.vel.cpu().numpy())
    _say("[md nvt graph] 4 x 10 steps bitwise equal")


def test_md_nvt_bf16_extended_energy_bounded():
    s = synth.cubic_lattice(6, 2.3, 0.25, 4, 99)
    drifts = {}
    for prec in ("fp32", "bf16"):
        hp, w, s, masses, v0, md = _setup(prec, s=s, cfg="E", rebuild=4, t_target_K=300.0, tau_fs=20.0)
        log = md.run(100).cpu().numpy()
        th = md.thermostat_log.cpu().numpy()
        h = log.sum(1) + th
        drift = np.abs(h - h[0]).max() / s.n_atoms
        moved = np.abs(th - th[0]).max() / s.n_atoms
        drifts[prec] = drift
        _say(f"[md nvt {prec}] 100 steps: max |H'(t)-H'(0)|/N = {drift * 1e3:.4f} meV/atom; "
             f"thermostat moved {moved * 1e3:.1f} meV/atom")
        assert moved > 5 * drift
        assert md.calc.status() == 0
    # as in the NVE test: the BF16 potential energy's evaluation error, up to
    # the energy gate at t and at 0, on top of a few times the FP32 drift
    assert drifts["bf16"] <= 5.0 * drifts["fp32"] + 2 * BF16_E_GATE


def test_md_nvt_rejects_missing_thermostat_state():
    import paper_2502_06073_amd as afm
    _, _, _, _, _, md = _setup("fp32", t_target_K=300.0, tau_fs=10.0)
    md.state.nh = None
    with pytest.raises(afm.AfmError):
        md.run(1)
    md.state.nh = md.nh.data_ptr()
    md.state.tau_fs = 0.0
    with pytest.raises(afm.AfmError):
        md.run(1)
