"""GPU training pieces: the Adam update against the oracle's, weight
replacement against a freshly created model, and a short optimisation of
the 8:1:1 energy/force/stress loss."""

import sys

import numpy as np
import pytest

import synth
from gpu_helpers import gpu_run, weights_for

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_adam_step_matches_oracle():
    import torch
    import paper_2502_06073_amd as afm
    from paper_2502_06073_amd import _abi
    from oracle import optim
    rng = np.random.default_rng(11)
    n = 100_003                      # several blocks and a ragged tail
    th0 = rng.standard_normal(n)
    grads = rng.standard_normal((5, n)).astype(np.float32)
    dev = "cuda"
    th = torch.tensor(th0, device=dev)
    m1 = torch.zeros(n, dtype=torch.float64, device=dev)
    m2 = torch.zeros(n, dtype=torch.float64, device=dev)
    ref = (th0.copy(), np.zeros(n), np.zeros(n))
    lib = _abi.load()
    for t in range(1, 6):
        g = torch.tensor(grads[t - 1], device=dev)
        _abi.check("afm_adam_step", lib.afm_adam_step(th.data_ptr(), g.data_ptr(), m1.data_ptr(), m2.data_ptr(), n,
                                                      1e-2, 0.9, 0.999, 1e-8, t, None))
        ref = optim.adam_step(ref[0], grads[t - 1].astype(np.float64), ref[1], ref[2], t, lr=1e-2)
    torch.cuda.synchronize()
    for got, want in zip((th, m1, m2), ref):
        np.testing.assert_allclose(got.cpu().numpy(), want, rtol=1e-12, atol=1e-15)
    _say("[adam] 5 steps on 100,003 parameters equal to the oracle to 1e-12")
    with pytest.raises(afm.AfmError):
        _abi.check("afm_adam_step", lib.afm_adam_step(th.data_ptr(), g.data_ptr(), m1.data_ptr(), m2.data_ptr(),
                                                      n, 1e-2, 0.9, 0.999, 1e-8, 0, None))


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_set_weights_equals_a_fresh_model(prec):
    import torch
    import paper_2502_06073_amd as afm
    hp = synth.load_hparams("B")
    s = synth.cubic_lattice(5, 2.2, 0.25, 4, 91)
    w1, w2 = weights_for(hp, 41), weights_for(hp, 42)
    fresh = gpu_run(hp, w2, s, prec)
    model = afm.Model(hp, w1, precision=prec)
    model.set_weights(w2)
    calc = afm.Calculator(model, afm.DeviceSystem.from_synth(s), r_list=hp["r_cut"])
    calc.build_neighbors()
    out = calc.energy_forces()
    torch.cuda.synchronize()
    for k in ("e_atom", "forces", "virial"):
        np.testing.assert_array_equal(out[k].cpu().numpy(), fresh[k])
    with pytest.raises(afm.AfmError):
        model.set_weights(w2[:-1])


def test_adam_lowers_the_stress_loss():
    import torch
    import paper_2502_06073_amd as afm
    from oracle import model as M
    hp = synth.load_hparams("C")
    s = synth.mixed_batch(4, 20, 40, 0.1, 10, 114)
    w = weights_for(hp, 43)
    e_hat, f_hat = synth.training_targets(s, 10)
    s_hat = synth.stress_targets(s, 11)
    model = afm.Model(hp, w, precision="fp32")
    calc = afm.Calculator(model, afm.DeviceSystem.from_synth(s), r_list=hp["r_cut"], second_order=True)
    opt = afm.Adam(model, w, lr=1e-3)
    dev = "cuda"
    n_s = torch.tensor(np.diff(s.seg), dtype=torch.float64, device=dev)
    per = np.asarray(s.pbc, dtype=bool)
    vol = torch.tensor([M.cell_volume(s.cell[k]) if per[k] else 1.0 for k in range(s.n_struct)], device=dev)
    mask = torch.tensor(per, device=dev, dtype=torch.float64)[:, None, None]
    losses = []
    for it in range(8):
        calc.build_neighbors()
        theta = torch.zeros(w.shape[0], dtype=torch.float64, requires_grad=True)
        E, F, W = afm.energy_forces_for_training(calc, theta, virial=True)
        de = (E - torch.tensor(e_hat, device=dev)) / n_s
        df = F - torch.tensor(f_hat, device=dev)
        ds = (W / vol[:, None, None] - torch.tensor(s_hat, device=dev)) * mask
        loss = 8.0 * (de * de).mean() + (df * df).sum() / (3.0 * s.n_atoms) + (ds * ds).sum() / (9.0 * per.sum())
        loss.backward()
        losses.append(loss.item())
        opt.step(theta.grad)
    _say(f"[adam train] loss {losses[0]:.4f} -> {losses[-1]:.4f} in {len(losses)} steps")
    assert losses[-1] < losses[0]
    # the starting loss against the oracle's
    ref = M.loss_and_grad(M.HParams.from_dict(hp), w, s, e_hat, f_hat, s_hat=s_hat, weights_efs=(8.0, 1.0, 1.0))
    assert abs(losses[0] - ref["loss"]) < 1e-5 * abs(ref["loss"])
