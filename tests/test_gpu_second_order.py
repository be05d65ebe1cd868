"""GPU double backward (weight gradients of force matching) against the
FP64 oracle's double backward (itself pinned by finite differences), and the
training loss gradient end to end through the autograd binding."""

import sys

import numpy as np
import pytest

import synth
from gpu_helpers import weights_for, weights_nonunit

pytestmark = pytest.mark.gpu
TOL = 1e-5          # FP32 relative norm


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _calc(hp, w, s, precision="fp32"):
    import paper_2502_06073_amd as afm
    model = afm.Model(hp, w, precision=precision)
    sysd = afm.DeviceSystem.from_synth(s)
    calc = afm.Calculator(model, sysd, r_list=hp.get("r_list", hp["r_cut"]), second_order=True)
    calc.build_neighbors()
    return calc


CASES = {
    "A": lambda: (synth.load_hparams("A"), synth.config_a()),
    "C_6clusters": lambda: (synth.load_hparams("C"), synth.clusters(6, 20, 80, 0.1, 0.9, 10, 111)),
    "C_periodic_small": lambda: (synth.load_hparams("C"), synth.cubic_lattice(4, 2.4, 0.2, 10, 112)),
}


@pytest.mark.parametrize("name", list(CASES))
def test_second_order_matches_oracle(name):
    import torch
    from oracle import model as M
    hp, s = CASES[name]()
    w = weights_for(hp, 31)
    rng = np.random.default_rng(3)
    gE = rng.standard_normal(s.n_struct)
    gF = rng.standard_normal((s.n_atoms, 3))
    calc = _calc(hp, w, s)
    g = calc.forces_backward(torch.tensor(gE, device="cuda"), torch.tensor(gF, device="cuda"))
    torch.cuda.synchronize()
    g = g.cpu().numpy().astype(np.float64)
    ref = M.vjp_weights(M.HParams.from_dict(hp), w, s, gE, gF)["grad_weights"]
    err = np.linalg.norm(g - ref) / np.linalg.norm(ref)
    lay = M.param_layout(M.HParams.from_dict(hp))
    worst, off = [], 0
    for b in lay:
        seg = slice(off, off + b["size"])
        den = max(np.linalg.norm(ref[seg]), 1e-30)
        worst.append((np.linalg.norm(g[seg] - ref[seg]) / den, b["name"]))
        off += b["size"]
    worst.sort(reverse=True)
    _say(f"[d2] {name}: rel {err:.2e}; worst blocks {worst[:3]}")
    assert err < TOL
    assert worst[0][0] < 10 * TOL


def test_second_order_force_term_only_and_energy_term_only():
    import torch
    from oracle import model as M
    hp, s = CASES["C_6clusters"]()
    w = weights_for(hp, 32)
    calc = _calc(hp, w, s)
    rng = np.random.default_rng(4)
    gE = rng.standard_normal(s.n_struct)
    gF = rng.standard_normal((s.n_atoms, 3))
    ge_only = calc.forces_backward(torch.tensor(gE, device="cuda"), None).cpu().numpy()
    gf_only = calc.forces_backward(None, torch.tensor(gF, device="cuda")).cpu().numpy()
    both = calc.forces_backward(torch.tensor(gE, device="cuda"), torch.tensor(gF, device="cuda")).cpu().numpy()
    np.testing.assert_allclose(ge_only + gf_only, both, rtol=1e-4, atol=1e-6 * np.abs(both).max())
    ref = M.vjp_weights(M.HParams.from_dict(hp), w, s, gE, np.zeros_like(gF))["grad_weights"]
    assert np.linalg.norm(ge_only - ref) / np.linalg.norm(ref) < TOL


def test_training_loss_gradient_through_autograd():
    import torch
    import paper_2502_06073_amd as afm
    from oracle import model as M
    hp, s = CASES["C_6clusters"]()
    w = weights_for(hp, 33)
    e_hat, f_hat = synth.training_targets(s, 5)
    calc = _calc(hp, w, s)
    theta = torch.zeros(w.shape[0], dtype=torch.float64, requires_grad=True)
    E, F = afm.energy_forces_for_training(calc, theta)
    n_s = torch.tensor(np.diff(s.seg), dtype=torch.float64, device="cuda")
    de = (E - torch.tensor(e_hat, device="cuda")) / n_s
    df = F - torch.tensor(f_hat, device="cuda")
    loss = (de * de).mean() + (df * df).sum() / (3.0 * s.n_atoms)
    loss.backward()
    ref = M.loss_and_grad(M.HParams.from_dict(hp), w, s, e_hat, f_hat)
    g = theta.grad.cpu().numpy()
    err = np.linalg.norm(g - ref["grad_weights"]) / np.linalg.norm(ref["grad_weights"])
    _say(f"[train] loss gpu {loss.item():.6f} oracle {ref['loss']:.6f}; grad rel {err:.2e}")
    assert abs(loss.item() - ref["loss"]) < 1e-5 * abs(ref["loss"])
    assert err < TOL


def _mixed():
    return synth.load_hparams("C"), synth.mixed_batch(4, 20, 60, 0.1, 10, 113)


def test_second_order_virial_term_matches_oracle():
    import torch
    from oracle import model as M
    hp, s = _mixed()
    w = weights_for(hp, 34)
    rng = np.random.default_rng(6)
    gE = rng.standard_normal(s.n_struct)
    gF = rng.standard_normal((s.n_atoms, 3))
    gW = rng.standard_normal((s.n_struct, 3, 3))
    calc = _calc(hp, w, s)
    dev = "cuda"
    g_all = calc.forces_backward(torch.tensor(gE, device=dev), torch.tensor(gF, device=dev),
                                 torch.tensor(gW, device=dev)).cpu().numpy().astype(np.float64)
    g_w = calc.forces_backward(None, None, torch.tensor(gW, device=dev)).cpu().numpy().astype(np.float64)
    ref_all = M.vjp_weights(M.HParams.from_dict(hp), w, s, gE, gF, grad_virial=gW)["grad_weights"]
    ref_w = M.vjp_weights(M.HParams.from_dict(hp), w, s, np.zeros(s.n_struct), np.zeros_like(gF),
                          grad_virial=gW)["grad_weights"]
    e_all = np.linalg.norm(g_all - ref_all) / np.linalg.norm(ref_all)
    e_w = np.linalg.norm(g_w - ref_w) / np.linalg.norm(ref_w)
    _say(f"[d2 virial] mixed batch {s.n_struct} structures / {s.n_atoms} atoms: all terms rel {e_all:.2e}, "
         f"virial term alone rel {e_w:.2e}")
    assert e_all < TOL and e_w < TOL


def test_training_loss_with_stress_through_autograd():
    """The 8:1:1 per-atom energy / force / stress loss (stress on the periodic
    structures) and its weight gradient, against the oracle."""
    import torch
    import paper_2502_06073_amd as afm
    from oracle import model as M
    hp, s = _mixed()
    w = weights_for(hp, 35)
    e_hat, f_hat = synth.training_targets(s, 8)
    s_hat = synth.stress_targets(s, 9)
    calc = _calc(hp, w, s)
    theta = torch.zeros(w.shape[0], dtype=torch.float64, requires_grad=True)
    E, F, W = afm.energy_forces_for_training(calc, theta, virial=True)
    dev = "cuda"
    n_s = torch.tensor(np.diff(s.seg), dtype=torch.float64, device=dev)
    per = np.asarray(s.pbc, dtype=bool)
    vol = torch.tensor([M.cell_volume(s.cell[k]) if per[k] else 1.0 for k in range(s.n_struct)], device=dev)
    mask = torch.tensor(per, device=dev, dtype=torch.float64)[:, None, None]
    de = (E - torch.tensor(e_hat, device=dev)) / n_s
    df = F - torch.tensor(f_hat, device=dev)
    ds = (W / vol[:, None, None] - torch.tensor(s_hat, device=dev)) * mask
    loss = 8.0 * (de * de).mean() + (df * df).sum() / (3.0 * s.n_atoms) + (ds * ds).sum() / (9.0 * per.sum())
    loss.backward()
    ref = M.loss_and_grad(M.HParams.from_dict(hp), w, s, e_hat, f_hat, s_hat=s_hat, weights_efs=(8.0, 1.0, 1.0))
    g = theta.grad.cpu().numpy()
    err = np.linalg.norm(g - ref["grad_weights"]) / np.linalg.norm(ref["grad_weights"])
    _say(f"[train stress] loss gpu {loss.item():.6f} oracle {ref['loss']:.6f}; grad rel {err:.2e}")
    assert abs(loss.item() - ref["loss"]) < 1e-5 * abs(ref["loss"])
    assert err < TOL


def test_second_order_nonunit_alpha_sigma():
    """Path-mixing weights alpha and species scales sigma_Z away from 1: their
    own gradient blocks and everything downstream of them."""
    import torch
    from oracle import model as M
    hp, s = CASES["C_6clusters"]()
    w = weights_nonunit(hp, 33)
    rng = np.random.default_rng(4)
    gE = rng.standard_normal(s.n_struct)
    gF = rng.standard_normal((s.n_atoms, 3))
    calc = _calc(hp, w, s)
    g = calc.forces_backward(torch.tensor(gE, device="cuda"), torch.tensor(gF, device="cuda"))
    torch.cuda.synchronize()
    g = g.cpu().numpy().astype(np.float64)
    ref = M.vjp_weights(M.HParams.from_dict(hp), w, s, gE, gF)["grad_weights"]
    err = np.linalg.norm(g - ref) / np.linalg.norm(ref)
    off, errs = 0, {}
    for b in M.param_layout(M.HParams.from_dict(hp)):
        seg = slice(off, off + b["size"])
        if b["name"].endswith(".alpha") or b["name"] == "species.scale":
            errs[b["name"]] = np.linalg.norm(g[seg] - ref[seg]) / max(np.linalg.norm(ref[seg]), 1e-30)
        off += b["size"]
    _say(f"[d2 alpha/sigma] rel {err:.2e}; {errs}")
    assert err < TOL
    assert max(errs.values()) < 10 * TOL


@pytest.mark.parametrize("name", ["A", "mixed", "C_periodic_small"])
def test_second_order_position_gradient_matches_oracle(name):
    """grad_pos = dJ/dr of J = sum gE E + sum gF . F + sum gW : W (second
    derivatives of the energy, incl. those of the edge basis), against the
    oracle's double backward with respect to the positions; the weight
    gradient of the same call is unchanged."""
    import torch
    from oracle import model as M
    if name == "mixed":
        hp, s = _mixed()
    else:
        hp, s = CASES[name]()
    w = weights_nonunit(hp, 36)
    rng = np.random.default_rng(7)
    gE = rng.standard_normal(s.n_struct)
    gF = rng.standard_normal((s.n_atoms, 3))
    gW = rng.standard_normal((s.n_struct, 3, 3))
    calc = _calc(hp, w, s)
    dev = "cuda"
    g, gp = calc.forces_backward(torch.tensor(gE, device=dev), torch.tensor(gF, device=dev),
                                 torch.tensor(gW, device=dev), want_pos=True)
    g_only = calc.forces_backward(torch.tensor(gE, device=dev), torch.tensor(gF, device=dev),
                                  torch.tensor(gW, device=dev))
    torch.cuda.synchronize()
    gp = gp.cpu().numpy()
    ref = M.vjp_weights(M.HParams.from_dict(hp), w, s, gE, gF, grad_virial=gW, want_pos=True)
    err = np.linalg.norm(gp - ref["grad_pos"]) / np.linalg.norm(ref["grad_pos"])
    errw = np.linalg.norm(g.cpu().numpy() - ref["grad_weights"]) / np.linalg.norm(ref["grad_weights"])
    _say(f"[d2 pos] {name}: {s.n_atoms} atoms, grad_pos rel {err:.2e} (|ref| {np.linalg.norm(ref['grad_pos']):.3e}), "
         f"weights rel {errw:.2e}")
    assert err < TOL
    assert errw < TOL
    np.testing.assert_array_equal(g.cpu().numpy(), g_only.cpu().numpy())
    assert calc.status() == 0


TOL_BF16 = 1.5e-2   # relative norm of the weight gradient with BF16 MFMA GEMMs (measured 3.0e-3 - 4.2e-3)


@pytest.mark.parametrize("name", ["C_6clusters", "C_periodic_small"])
def test_second_order_bf16_gemms_match_oracle(name):
    """BF16 models run the double backward's GEMMs on BF16 MFMA (operands
    rounded to bf16, FP32 accumulation): the weight gradient against the
    FP64 oracle's, overall and per parameter block."""
    import torch
    from oracle import model as M
    hp, s = CASES[name]()
    w = weights_nonunit(hp, 33)
    rng = np.random.default_rng(4)
    gE = rng.standard_normal(s.n_struct)
    gF = rng.standard_normal((s.n_atoms, 3))
    calc = _calc(hp, w, s, precision="bf16")
    g = calc.forces_backward(torch.tensor(gE, device="cuda"), torch.tensor(gF, device="cuda"))
    torch.cuda.synchronize()
    g = g.cpu().numpy().astype(np.float64)
    ref = M.vjp_weights(M.HParams.from_dict(hp), w, s, gE, gF)["grad_weights"]
    err = np.linalg.norm(g - ref) / np.linalg.norm(ref)
    cos = float(g @ ref / (np.linalg.norm(g) * np.linalg.norm(ref)))
    lay = M.param_layout(M.HParams.from_dict(hp))
    worst, off = [], 0
    for b in lay:
        seg = slice(off, off + b["size"])
        den = max(np.linalg.norm(ref[seg]), 1e-30)
        worst.append((round(float(np.linalg.norm(g[seg] - ref[seg]) / den), 5), b["name"]))
        off += b["size"]
    worst.sort(reverse=True)
    _say(f"[d2 bf16] {name}: rel {err:.2e}, cosine {cos:.6f}; worst blocks {worst[:4]}")
    assert err < TOL_BF16 and cos > 0.999
