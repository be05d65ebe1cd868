"""The fused last latent layer (forward and adjoint in one kernel) against
the separate kernels: energies, forces and virials bitwise equal through
afm_energy_forces, for 2- and 3-layer models, the exact and the fast
adjoint, on inputs spanning several tiles with ragged tails; where it is
built and where not."""

import sys

import numpy as np
import pytest

import synth
from gpu_helpers import weights_nonunit

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


CASES = {
    "Bshape_7cube": lambda: (synth.load_hparams("B"), synth.cubic_lattice(7, 2.2, 0.25, 4, 171)),
    "D_12mixed": lambda: (synth.load_hparams("D"), synth.config_d(12)),
}


@pytest.mark.parametrize("prec", ["bf16", "bf16_fast"])
@pytest.mark.parametrize("name", list(CASES))
def test_fused_last_layer_bitwise_equal(name, prec):
    import torch
    import paper_2502_06073_amd as afm
    hp, s = CASES[name]()
    w = weights_nonunit(hp, 172)
    model = afm.Model(hp, w, precision=prec)
    calc = afm.Calculator(model, afm.DeviceSystem.from_synth(s))
    calc.build_neighbors()
    res = {}
    for on in (True, False):
        assert model.set_fused_last(on) == on
        out = calc.energy_forces()
        torch.cuda.synchronize()
        res[on] = {k: v.cpu().numpy() for k, v in out.items()}
    for k in ("e_atom", "e_struct", "forces", "virial"):
        np.testing.assert_array_equal(res[True][k], res[False][k], err_msg=k)
    _say(f"[fused {prec}] {name}: fused == separate bitwise ({s.n_atoms} atoms)")
    assert calc.status() == 0


def test_fused_last_layer_where_built():
    import paper_2502_06073_amd as afm
    hp, s = CASES["Bshape_7cube"]()
    w = weights_nonunit(hp, 173)
    m16 = afm.Model(hp, w, precision="bf16")
    assert m16.set_fused_last(True)
    m16.set_edge_tile(128, 16)
    assert not m16.set_fused_last(True)          # 64-edge tiles only
    m32 = afm.Model(hp, w, precision="fp32")
    assert not m32.set_fused_last(True)          # BF16 chains only
