"""CPU-side checks of the C-ABI library: it loads, exports every entry point
the header declares, its host-side tables (weight layout, real CG tensors)
agree with the oracle's independent derivations, and argument errors come
back as status codes (no GPU call is made by these paths)."""

import ctypes as C
import os
import re

import numpy as np
import pytest

import synth
from oracle import model as M
from oracle import so3

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
afm = pytest.importorskip("paper_2502_06073_amd")
from paper_2502_06073_amd import _abi  # noqa: E402


def _lib():
    if not os.path.exists(_abi.LIB_PATH):
        pytest.skip("libafm.so not built (python -m paper_2502_06073_amd.build)")
    return _abi.load()


def test_exports_every_declared_symbol():
    lib = _lib()
    hdr = open(os.path.join(ROOT, "include", "afm.h")).read()
    names = set(re.findall(r"\b(afm_[a-z_]+)\s*\(", hdr))
    assert len(names) >= 14
    for n in sorted(names):
        assert hasattr(lib, n), n
    assert set(_abi.EXPORTS) == names


@pytest.mark.parametrize("name", list("ABCDE"))
def test_param_layout_matches_oracle(name):
    _lib()
    hp = synth.load_hparams(name)
    ours = afm.param_layout(hp)
    ref = M.param_layout(M.HParams.from_dict(hp))
    assert [b["name"] for b in ours] == [b["name"] for b in ref]
    for a, b in zip(ours, ref):
        assert tuple(a["shape"]) == tuple(b["shape"]), a["name"]
        assert a["fan_in"] == b["fan_in"] and a["init"] == b["init"], a["name"]
    assert sum(b["size"] for b in ours) == M.n_params(M.HParams.from_dict(hp))


@pytest.mark.parametrize("lmax,nl,c", [(2, 2, 16), (2, 3, 8), (1, 3, 64), (0, 2, 32)])
def test_dense_mixing_layout_matches_oracle(lmax, nl, c):
    _lib()
    hp = dict(synth.load_hparams("A"), l_max=lmax, n_layers=nl, channels=c, mixing="dense")
    ours = afm.param_layout(hp)
    ref = M.param_layout(M.HParams.from_dict(hp))
    assert [b["name"] for b in ours] == [b["name"] for b in ref]
    for a, b in zip(ours, ref):
        assert tuple(a["shape"]) == tuple(b["shape"]), a["name"]
        assert a["fan_in"] == b["fan_in"] and a["init"] == b["init"], a["name"]
    assert any(b["name"].endswith(".mix") for b in ours)
    assert not any(b["name"].endswith(".alpha") for b in ours)


def test_dense_mixing_refusals():
    lib = _lib()
    hp = synth.load_hparams("A")
    nb, npar = C.c_int64(), C.c_int64()
    for kw, code in ((dict(mixing="dense", l_max=3, channels=16, n_layers=2), -4),
                     (dict(mixing="dense", channels=128), -4)):
        bad = afm.hparams_struct(dict(hp, **kw))
        assert lib.afm_param_layout_size(C.byref(bad), C.byref(nb), C.byref(npar)) == code, kw
    h = afm.hparams_struct(hp)
    h.mixing = 2
    assert lib.afm_param_layout_size(C.byref(h), C.byref(nb), C.byref(npar)) == -1
    with pytest.raises(ValueError):
        afm.hparams_struct(dict(hp, mixing="full"))


def test_table1_counts_through_library():
    _lib()
    want = {64: 46914, 256: 676466, 512: 2614194}
    for w, c, h in [(64, 16, 64), (256, 64, 128)]:
        hp = dict(n_species=89, l_max=2, n_layers=2, latent=w, channels=c, n_bessel=8, poly_p=6,
                  twobody=[w // 4, w // 2, w], latent_depth=3, edge_hidden=h, r_cut=5.2)
        assert sum(b["size"] for b in afm.param_layout(hp)) == want[w]


@pytest.mark.parametrize("t", [(l1, l2, l3) for l1 in range(4) for l2 in range(4)
                               for l3 in range(abs(l1 - l2), min(l1 + l2, 3) + 1)])
def test_cg_tables_match_oracle(t):
    _lib()
    np.testing.assert_allclose(afm.cg_real(*t), so3.cg(*t), atol=1e-13)


def test_host_error_paths():
    lib = _lib()
    hp = synth.load_hparams("A")
    h = afm.hparams_struct(hp)
    out = C.c_void_p()
    w = np.zeros(10)
    rc = lib.afm_model_create(C.byref(h), w.ctypes.data_as(C.POINTER(C.c_double)), 10, 1, C.byref(out))
    assert rc == -6 and out.value is None           # AFM_E_WEIGHTS
    assert b"expected 4836" in lib.afm_last_error()
    rc = lib.afm_model_create(C.byref(h), w.ctypes.data_as(C.POINTER(C.c_double)), 10, 0, C.byref(out))
    assert rc == -4                                 # FP64 on the device is not built
    rc = lib.afm_model_create(None, None, 0, 1, C.byref(out))
    assert rc == -1
    nb, npar = C.c_int64(), C.c_int64()
    for kw in (dict(l_max=4), dict(l_max=3),                       # l = 4; 8 channels at l = 3
               dict(l_max=3, channels=16, n_layers=3)):            # three layers at l = 3
        bad = afm.hparams_struct(dict(hp, **kw))
        assert lib.afm_param_layout_size(C.byref(bad), C.byref(nb), C.byref(npar)) == -4, kw
    ok = afm.hparams_struct(dict(hp, l_max=3, channels=16, n_layers=2))
    assert lib.afm_param_layout_size(C.byref(ok), C.byref(nb), C.byref(npar)) == 0
    assert npar.value == M.n_params(M.HParams.from_dict(dict(hp, l_max=3, channels=16, n_layers=2,
                                                              avg_num_neighbors=1.0, energy_scale=1.0)))
    bad = afm.hparams_struct(dict(hp, twobody=[16, 48]))
    assert lib.afm_param_layout_size(C.byref(bad), C.byref(nb), C.byref(npar)) == -1
    ws = _abi.Workspace()
    assert lib.afm_workspace_plan(None, 10, 1, 100, 0, 0, None) == -1
    assert lib.afm_workspace_plan(None, 10, 0, 100, 0, 0, C.byref(ws)) == -1
    assert lib.afm_workspace_plan(None, 10, 1, 100, 0, 0, C.byref(ws)) == 0 and ws.bytes > 0
    assert lib.afm_build_neighbors(None, 4.0, None, None, None) == -1
    assert lib.afm_strerror(-2) == b"buffer capacity exceeded"
    assert lib.afm_version().startswith(b"afm")
    nanw = synth.draw_weights(M.param_layout(M.HParams.from_dict(hp)), 1)
    nanw[3] = np.nan
    rc = lib.afm_model_create(C.byref(h), nanw.ctypes.data_as(C.POINTER(C.c_double)), nanw.shape[0], 1,
                              C.byref(out))
    assert rc == -3                                 # AFM_E_NONFINITE


def test_stage_costs_cover_traced_stages():
    """The cost model names every traced stage of energy_forces and its MLP
    figures equal the multiply-adds of the layer widths."""
    import paper_2502_06073_amd as afm
    hp = synth.load_hparams("B")
    c = afm.stage_costs(hp)
    names = {"geometry", "twobody_fwd", "twobody_bwd", "geometry_bwd", "energy", "force_scatter"}
    for L in (1, 2):
        names |= {f"tp_fwd{L}", f"tp_bwd{L}", f"latent_fwd{L}", f"latent_bwd{L}"}
    names.add("latent_fb2")                  # the fused last layer: forward + adjoint
    names.add("second_order")                # the double backward's GEMMs
    assert set(c) == names
    assert c["latent_fb2"]["flops_per_edge"] == c["latent_fwd2"]["flops_per_edge"] + c["latent_bwd2"]["flops_per_edge"]
    W, C, D = hp["latent"], hp["channels"], hp["latent_depth"]
    env = (hp["l_max"] + 1) * C
    lat1 = (W + 3 * C) * W + (D - 1) * W * W
    assert c["latent_fwd1"]["flops_per_edge"] == 2 * (lat1 + W * env)
    assert c["latent_fwd2"]["flops_per_edge"] == 2 * (lat1 + W)
    assert c["latent_bwd2"]["flops_per_edge"] == 2 * lat1
    tb = hp["twobody"]
    assert c["twobody_fwd"]["flops_per_edge"] == 2 * (hp["n_bessel"] * tb[0] + tb[0] * tb[1] + tb[1] * tb[2] + W * env)
    assert all(v["kind"] == ("mfma" if k.startswith(("latent", "twobody", "second")) else "vector") for k, v in c.items())
    # the double backward: three products (forward, input and weight gradient) per weight matrix over
    # two stacked rows per edge, two for the first two-body layer
    lat = sum(3 * (((W + 3 * C) if k == 0 else W) * W) for k in range(D)) * 2 + 3 * W * env
    two = 2 * (2 * hp["n_species"] + hp["n_bessel"]) * tb[0] + 3 * (tb[0] * tb[1] + tb[1] * tb[2]) + 3 * W * env
    assert c["second_order"]["flops_per_edge"] == 4 * (lat + two)
    assert all(v["bytes_per_edge"] > 0 for v in c.values())


def test_stage_costs_dense_mixing():
    """With dense mixing the cost model names the mixing GEMMs of every layer
    below the last (FP32 matrix-core stages) and their flops are 2 c^2 per
    mixed product component."""
    import paper_2502_06073_amd as afm
    hp = dict(synth.load_hparams("B"), mixing="dense")
    c = afm.stage_costs(hp)
    assert {"mix_fwd1", "mix_bwd1"} <= set(c) and "mix_fwd2" not in c
    assert c["mix_fwd1"]["kind"] == "mfma_f32" and c["tp_fwd1"]["kind"] == "vector"
    paths, _, outs = M.path_sets(M.HParams.from_dict(hp))
    used = set(outs[0])
    comps = sum(2 * p[3] + 1 for p in paths[0] if (p[3], p[4]) in used)
    C_ = hp["channels"]
    assert c["mix_fwd1"]["flops_per_edge"] == 2 * C_ * C_ * comps == c["mix_bwd1"]["flops_per_edge"]


def test_stage_costs_lmax3():
    """The cost model of an l_max = 3 model (its CG tensors have up to 7^3
    entries) gives positive figures for every stage and more tensor-product
    work than the l_max = 2 model of the same widths."""
    import paper_2502_06073_amd as afm
    hp2 = synth.load_hparams("B")
    c2 = afm.stage_costs(hp2)
    c3 = afm.stage_costs(dict(hp2, l_max=3))
    assert set(c3) == set(c2)
    assert all(v["flops_per_edge"] > 0 and v["bytes_per_edge"] > 0 for v in c3.values())
    for k in ("tp_fwd1", "tp_bwd1", "tp_fwd2", "tp_bwd2"):
        assert c3[k]["flops_per_edge"] > c2[k]["flops_per_edge"], k
