"""afm_energy_forces_noalloc (the library's static device scratch in place of
a caller workspace) against afm_energy_forces with a caller workspace: two
calls in a row on one model, the second on a smaller system (the scratch
keeps the first call's contents), FP32 and BF16; and the size limit comes
back as AFM_E_CAPACITY without any device work."""

import ctypes as C
import sys

import numpy as np
import pytest

import synth
from gpu_helpers import rel, weights_nonunit

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _pair(model, s):
    import torch
    import paper_2502_06073_amd as afm
    calc = afm.Calculator(model, afm.DeviceSystem.from_synth(s))
    calc.build_neighbors()
    ref = calc.energy_forces()
    torch.cuda.synchronize()
    ref = {k: v.cpu().numpy() for k, v in ref.items()}
    out = calc.energy_forces_noalloc()
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy() for k, v in out.items()}
    assert calc.status() == 0
    return ref, out, int(calc.nl.n_edges.item())


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_noalloc_matches_workspace_entry_point(prec):
    import paper_2502_06073_amd as afm
    hp = synth.load_hparams("B")
    w = weights_nonunit(hp, 4242)
    model = afm.Model(hp, w, precision=prec)
    # 13,824 atoms (edges processed in several row chunks inside the static
    # scratch), then 512 atoms on the same model and the same scratch
    for n_side, seed in ((24, 5101), (8, 5102)):
        s = synth.cubic_lattice(n_side, 2.2, 0.25, 4, seed)
        _say(f"[noalloc {prec}] {s.n_atoms} atoms")
        ref, out, ne = _pair(model, s)
        errs = {k: rel(out[k], ref[k]) for k in ("e_atom", "e_struct", "forces", "virial")}
        same = all(np.array_equal(out[k], ref[k]) for k in errs)
        _say(f"[noalloc {prec}] {s.n_atoms} atoms, {ne} edges: rel err {errs}; bitwise equal {same}")
        for k, e in errs.items():
            assert e <= 1e-5, (k, e)


def test_noalloc_rejects_oversize_system():
    import paper_2502_06073_amd as afm
    from paper_2502_06073_amd import _abi
    hp = synth.load_hparams("B")
    w = weights_nonunit(hp, 4243)
    model = afm.Model(hp, w, precision="bf16")
    s = synth.cubic_lattice(4, 2.2, 0.25, 4, 5103)
    calc = afm.Calculator(model, afm.DeviceSystem.from_synth(s))
    nl = calc.nl.struct()
    nl.capacity = 2_000_000_000     # edge arrays alone exceed the scratch: rejected on the host
    out = calc._outs(True)
    lib = _abi.load()
    import torch
    with torch.cuda.device(model.device):
        rc = lib.afm_energy_forces_noalloc(model.handle, C.byref(calc.sysd.struct()), C.byref(nl),
                                           out[0].data_ptr(), out[1].data_ptr(), out[2].data_ptr(),
                                           out[3].data_ptr(), None)
    msg = lib.afm_last_error().decode()
    _say(f"[noalloc] oversize -> {rc}: {msg}")
    assert rc == -2 and "static scratch" in msg
