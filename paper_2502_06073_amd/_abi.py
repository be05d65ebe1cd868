"""ctypes declarations of the C ABI in include/afm.h (marshalling only)."""

from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libafm.so")

AFM_OK = 0
STATUS = {0: "AFM_OK", -1: "AFM_E_INVALID", -2: "AFM_E_CAPACITY", -3: "AFM_E_NONFINITE",
          -4: "AFM_E_UNSUPPORTED", -5: "AFM_E_HIP", -6: "AFM_E_WEIGHTS"}
FLAG_CAPACITY, FLAG_NONFINITE, FLAG_SPECIES, FLAG_SKIN, FLAG_IMAGES = 1, 2, 4, 8, 16
PRECISION = {"fp64": 0, "fp32": 1, "bf16": 2, "bf16_fast": 3}
STATIC_SCRATCH_BYTES = 256 << 20   # AFM_STATIC_SCRATCH_BYTES
TILE_SHAPES = ((64, 8), (128, 16), (128, 8))   # edge-tile shapes, in the tuner's order


class Hparams(C.Structure):
    _fields_ = [("n_species", C.c_int32), ("l_max", C.c_int32), ("n_layers", C.c_int32),
                ("latent", C.c_int32), ("channels", C.c_int32), ("n_bessel", C.c_int32),
                ("poly_p", C.c_int32), ("n_twobody", C.c_int32), ("twobody", C.c_int32 * 4),
                ("latent_depth", C.c_int32), ("edge_hidden", C.c_int32), ("r_cut", C.c_double),
                ("avg_num_neighbors", C.c_double), ("energy_scale", C.c_double),
                ("mixing", C.c_int32)]


class ParamBlock(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("offset", C.c_int64), ("rows", C.c_int64),
                ("cols", C.c_int64), ("fan_in", C.c_int64), ("init", C.c_int32)]


class System(C.Structure):
    _fields_ = [("n_atoms", C.c_int64), ("n_struct", C.c_int64), ("pos", C.c_void_p),
                ("species", C.c_void_p), ("cell", C.c_void_p), ("pbc", C.c_void_p),
                ("seg", C.c_void_p)]


class Nlist(C.Structure):
    _fields_ = [("capacity", C.c_int64), ("row_ptr", C.c_void_p), ("col", C.c_void_p),
                ("shift", C.c_void_p), ("rev", C.c_void_p), ("n_edges", C.c_void_p),
                ("status", C.c_void_p)]


class Workspace(C.Structure):
    _fields_ = [("ptr", C.c_void_p), ("bytes", C.c_int64), ("n_atoms", C.c_int64),
                ("n_struct", C.c_int64), ("edge_capacity", C.c_int64), ("chunk_edges", C.c_int64),
                ("n_chunks", C.c_int64), ("max_row", C.c_int64), ("precision", C.c_int32),
                ("with_second_order", C.c_int32)]


class TraceStat(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("launches", C.c_int32), ("total_ms", C.c_double)]


class StageCost(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("kind", C.c_int32), ("flops_per_edge", C.c_double),
                ("bytes_per_edge", C.c_double), ("bytes_per_atom", C.c_double)]


class MdState(C.Structure):
    _fields_ = [("pos", C.c_void_p), ("vel", C.c_void_p), ("forces", C.c_void_p),
                ("mass_by_species", C.c_void_p), ("dt_fs", C.c_double), ("skin", C.c_double),
                ("rebuild_every", C.c_int32), ("use_graph", C.c_int32), ("step", C.c_int64),
                ("energy_log", C.c_void_p),
                ("e_atom", C.c_void_p), ("e_struct", C.c_void_p),
                ("t_target_K", C.c_double), ("tau_fs", C.c_double), ("n_dof", C.c_int64),
                ("nh", C.c_void_p), ("thermostat_log", C.c_void_p)]


EXPORTS = {
    "afm_param_layout_size": [C.POINTER(Hparams), C.POINTER(C.c_int64), C.POINTER(C.c_int64)],
    "afm_param_layout_block": [C.POINTER(Hparams), C.c_int64, C.POINTER(ParamBlock)],
    "afm_cg_real": [C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_double)],
    "afm_model_create": [C.POINTER(Hparams), C.POINTER(C.c_double), C.c_int64, C.c_int,
                         C.POINTER(C.c_void_p)],
    "afm_model_destroy": [C.c_void_p],
    "afm_model_set_weights": [C.c_void_p, C.POINTER(C.c_double), C.c_int64],
    "afm_adam_step": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_double, C.c_double,
                      C.c_double, C.c_double, C.c_int64, C.c_void_p],
    "afm_workspace_plan": [C.c_void_p, C.c_int64, C.c_int64, C.c_int64, C.c_int64, C.c_int32,
                           C.POINTER(Workspace)],
    "afm_build_neighbors": [C.POINTER(System), C.c_double, C.POINTER(Nlist), C.POINTER(Workspace),
                            C.c_void_p],
    "afm_forward_energy": [C.c_void_p, C.POINTER(System), C.POINTER(Nlist), C.c_void_p, C.c_void_p,
                           C.POINTER(Workspace), C.c_void_p],
    "afm_backward_forces": [C.c_void_p, C.POINTER(System), C.POINTER(Nlist), C.c_void_p, C.c_void_p,
                            C.c_void_p, C.POINTER(Workspace), C.c_void_p],
    "afm_energy_forces": [C.c_void_p, C.POINTER(System), C.POINTER(Nlist), C.c_void_p, C.c_void_p,
                          C.c_void_p, C.c_void_p, C.POINTER(Workspace), C.c_void_p],
    "afm_energy_forces_noalloc": [C.c_void_p, C.POINTER(System), C.POINTER(Nlist), C.c_void_p, C.c_void_p,
                                  C.c_void_p, C.c_void_p, C.c_void_p],
    "afm_backward_forces_backward": [C.c_void_p, C.POINTER(System), C.POINTER(Nlist), C.c_void_p,
                                     C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(Workspace),
                                     C.c_void_p],
    "afm_set_edge_tile": [C.c_void_p, C.c_int32, C.c_int32],
    "afm_get_edge_tile": [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32)],
    "afm_set_fused_last": [C.c_void_p, C.c_int32, C.POINTER(C.c_int32)],
    "afm_tune_edge_tile": [C.c_void_p, C.POINTER(System), C.POINTER(Nlist), C.POINTER(Workspace), C.c_char_p,
                           C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_double),
                           C.POINTER(C.c_int32), C.c_void_p],
    "afm_md_step": [C.c_void_p, C.POINTER(System), C.POINTER(Nlist), C.POINTER(MdState), C.c_int32,
                    C.POINTER(Workspace), C.c_void_p],
    "afm_trace_enable": [C.c_int32],
    "afm_trace_read": [C.POINTER(TraceStat), C.c_int32, C.POINTER(C.c_int32)],
    "afm_stage_costs": [C.POINTER(Hparams), C.POINTER(StageCost), C.c_int32, C.POINTER(C.c_int32)],
    "afm_md_graph_count": [],
    "afm_strerror": [C.c_int],
    "afm_last_error": [],
    "afm_version": [],
}
RESTYPES = {"afm_md_graph_count": C.c_int64, "afm_strerror": C.c_char_p, "afm_last_error": C.c_char_p, "afm_version": C.c_char_p}

_LIB = None


def load(path: str = LIB_PATH) -> C.CDLL:
    """Load the built library; raises if it is missing (no fallback)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with "
                           "`python -m paper_2502_06073_amd.build`")
    lib = C.CDLL(path)
    for name, args in EXPORTS.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = RESTYPES.get(name, C.c_int)
    _LIB = lib
    return lib


class AfmError(RuntimeError):
    def __init__(self, fn: str, code: int):
        msg = load().afm_last_error().decode()
        super().__init__(f"{fn} -> {STATUS.get(code, code)}: {msg}")
        self.code = code


def check(fn: str, code: int):
    if code != AFM_OK:
        raise AfmError(fn, code)
