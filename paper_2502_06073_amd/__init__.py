"""MI355X (gfx950) library for the strictly-local equivariant edge potential
of Allegro-FM (arXiv 2502.06073): Python binding of the C ABI.

Every step of the computation runs in the HIP kernels of ``libafm.so``;
this module only marshals arguments.  PyTorch provides device memory and the
current HIP stream.  There is no CPU fallback: without the built library or
a GPU the calls raise.

    import paper_2502_06073_amd as afm
    model = afm.Model(hparams, weights, precision="bf16")
    sysd = afm.DeviceSystem.from_arrays(pos, species, cell, pbc, seg)
    calc = afm.Calculator(model, sysd, r_list=hparams["r_cut"])
    out = calc.energy_forces()        # e_atom, e_struct, forces, virial
"""

from __future__ import annotations

import ctypes as C
import sys
from typing import Dict, List, Optional

import numpy as np
import torch

from . import _abi
from ._abi import AfmError, check, load

__all__ = ["Model", "DeviceSystem", "NeighborList", "Workspace", "Calculator",
           "param_layout", "cg_real", "hparams_struct", "stage_costs", "energy_and_forces", "AfmError", "Adam",
           "trace_enable", "trace_read", "energy_forces_for_training", "MD", "EvalGraph"]


def trace_enable(on: bool = True) -> None:
    """Start (clearing old records) or stop per-stage HIP-event timing."""
    check("afm_trace_enable", load().afm_trace_enable(1 if on else 0))


def trace_read() -> Dict[str, Dict[str, float]]:
    """Per-stage launch counts and summed GPU milliseconds since trace_enable."""
    lib = load()
    n = C.c_int32()
    check("afm_trace_read", lib.afm_trace_read(None, 0, C.byref(n)))
    arr = (_abi.TraceStat * max(1, n.value))()
    check("afm_trace_read", lib.afm_trace_read(arr, n.value, C.byref(n)))
    return {arr[k].name.decode(): dict(launches=arr[k].launches, total_ms=arr[k].total_ms)
            for k in range(n.value)}


def stage_costs(hp: Dict) -> Dict[str, Dict[str, float]]:
    """Algorithmic flops/bytes per edge (and bytes per atom) of each traced
    stage of energy_forces for hyper-parameters `hp`, keyed like trace_read()."""
    lib = load()
    h = hparams_struct(hp)
    n = C.c_int32()
    check("afm_stage_costs", lib.afm_stage_costs(C.byref(h), None, 0, C.byref(n)))
    arr = (_abi.StageCost * max(1, n.value))()
    check("afm_stage_costs", lib.afm_stage_costs(C.byref(h), arr, n.value, C.byref(n)))
    return {arr[k].name.decode(): dict(kind={0: "mfma", 1: "vector", 2: "mfma_f32"}[arr[k].kind],
                                       flops_per_edge=arr[k].flops_per_edge,
                                       bytes_per_edge=arr[k].bytes_per_edge,
                                       bytes_per_atom=arr[k].bytes_per_atom)
            for k in range(n.value)}


def _stream_ptr(device) -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


# tensor-product output mixing: one weight per (path, channel), or a dense
# channel-mixing matrix per path
MIXING = {"path": 0, "dense": 1}


def hparams_struct(hp: Dict) -> _abi.Hparams:
    tb = list(hp["twobody"])
    h = _abi.Hparams()
    h.n_species = int(hp["n_species"])
    h.l_max = int(hp["l_max"])
    h.n_layers = int(hp["n_layers"])
    h.latent = int(hp["latent"])
    h.channels = int(hp["channels"])
    h.n_bessel = int(hp["n_bessel"])
    h.poly_p = int(hp["poly_p"])
    h.n_twobody = len(tb)
    for k in range(4):
        h.twobody[k] = int(tb[k]) if k < len(tb) else 0
    h.latent_depth = int(hp["latent_depth"])
    h.edge_hidden = int(hp["edge_hidden"])
    h.r_cut = float(hp["r_cut"])
    h.avg_num_neighbors = float(hp.get("avg_num_neighbors", 1.0))
    h.energy_scale = float(hp.get("energy_scale", 1.0))
    mixing = hp.get("mixing", "path")
    if mixing not in MIXING:
        raise ValueError(f"mixing must be one of {sorted(MIXING)}, not {mixing!r}")
    h.mixing = MIXING[mixing]
    return h


def param_layout(hp: Dict) -> List[Dict]:
    """The library's flat weight layout (block name, offset, shape, fan-in, init)."""
    lib = load()
    h = hparams_struct(hp)
    nb, npar = C.c_int64(), C.c_int64()
    check("afm_param_layout_size", lib.afm_param_layout_size(C.byref(h), C.byref(nb), C.byref(npar)))
    out = []
    for k in range(nb.value):
        b = _abi.ParamBlock()
        check("afm_param_layout_block", lib.afm_param_layout_block(C.byref(h), k, C.byref(b)))
        init = {0: "fan_in", 1: "normal", 2: "ones"}[b.init]
        shape = (b.rows,) if b.name.decode().startswith("species.") else (b.rows, b.cols)
        out.append(dict(name=b.name.decode(), offset=b.offset, shape=shape,
                        size=b.rows * b.cols, fan_in=b.fan_in, init=init))
    return out


def cg_real(l1: int, l2: int, l3: int) -> np.ndarray:
    lib = load()
    out = np.zeros((2 * l1 + 1) * (2 * l2 + 1) * (2 * l3 + 1))
    check("afm_cg_real", lib.afm_cg_real(l1, l2, l3, out.ctypes.data_as(C.POINTER(C.c_double))))
    return out.reshape(2 * l1 + 1, 2 * l2 + 1, 2 * l3 + 1)


class Model:
    """Device copy of a weight vector for one precision ("fp32", "bf16" or
    "bf16_fast", the BF16 path with the fast adjoint)."""

    def __init__(self, hp: Dict, weights: np.ndarray, precision: str = "bf16", device: int = 0):
        lib = load()
        self.hp = dict(hp)
        self.precision = precision
        self.device = torch.device("cuda", device)
        w = np.ascontiguousarray(weights, dtype=np.float64)
        h = hparams_struct(hp)
        handle = C.c_void_p()
        with torch.cuda.device(self.device):
            check("afm_model_create",
                  lib.afm_model_create(C.byref(h), w.ctypes.data_as(C.POINTER(C.c_double)), w.shape[0],
                                       _abi.PRECISION[precision], C.byref(handle)))
        self.handle = handle

    def set_weights(self, weights: np.ndarray):
        """New weight values (same layout); synchronises the device."""
        w = np.ascontiguousarray(weights, dtype=np.float64)
        with torch.cuda.device(self.device):
            check("afm_model_set_weights",
                  load().afm_model_set_weights(self.handle, w.ctypes.data_as(C.POINTER(C.c_double)), w.shape[0]))

    @property
    def edge_tile(self):
        """(edges, wavefronts) per workgroup tile of the BF16 MLP chains
        ((0, 0) for FP32)."""
        e, w = C.c_int32(), C.c_int32()
        check("afm_get_edge_tile", load().afm_get_edge_tile(self.handle, C.byref(e), C.byref(w)))
        return int(e.value), int(w.value)

    def set_edge_tile(self, edges: int, waves: int):
        check("afm_set_edge_tile", load().afm_set_edge_tile(self.handle, int(edges), int(waves)))

    def set_fused_last(self, on: bool) -> bool:
        """Fused last-layer forward + adjoint in energy_forces (default on);
        returns whether the model's current shape uses it."""
        active = C.c_int32()
        check("afm_set_fused_last", load().afm_set_fused_last(self.handle, int(bool(on)), C.byref(active)))
        return bool(active.value)

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            with torch.cuda.device(self.device):
                load().afm_model_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        # during interpreter shutdown torch's operator registry may already be
        # gone, and the device context in close() would abort the process;
        # the driver releases the device memory at exit anyway
        if sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


class DeviceSystem:
    """Device tensors of a batch of structures (see afm_system)."""

    def __init__(self, pos, species, cell, pbc, seg):
        self.pos, self.species, self.cell, self.pbc, self.seg = pos, species, cell, pbc, seg

    @staticmethod
    def from_arrays(pos, species, cell, pbc, seg, device="cuda:0") -> "DeviceSystem":
        dev = torch.device(device)
        return DeviceSystem(
            torch.as_tensor(np.ascontiguousarray(pos, np.float64), device=dev),
            torch.as_tensor(np.ascontiguousarray(species, np.int32), device=dev),
            torch.as_tensor(np.ascontiguousarray(np.asarray(cell, np.float64).reshape(-1, 3, 3)), device=dev),
            torch.as_tensor(np.ascontiguousarray(pbc, np.uint8), device=dev),
            torch.as_tensor(np.ascontiguousarray(seg, np.int64), device=dev))

    @staticmethod
    def from_synth(s, device="cuda:0") -> "DeviceSystem":
        return DeviceSystem.from_arrays(s.pos, s.species, s.cell, s.pbc, s.seg, device)

    @property
    def n_atoms(self) -> int:
        return int(self.pos.shape[0])

    @property
    def n_struct(self) -> int:
        return int(self.seg.shape[0] - 1)

    def struct(self, pos: Optional[torch.Tensor] = None) -> _abi.System:
        s = _abi.System()
        s.n_atoms = self.n_atoms
        s.n_struct = self.n_struct
        s.pos = _ptr(self.pos if pos is None else pos)
        s.species = _ptr(self.species)
        s.cell = _ptr(self.cell)
        s.pbc = _ptr(self.pbc)
        s.seg = _ptr(self.seg)
        return s


class NeighborList:
    """Device CSR edge list with a fixed edge capacity."""

    def __init__(self, n_atoms: int, capacity: int, device):
        self.capacity = int(capacity)
        self.row_ptr = torch.zeros(n_atoms + 1, dtype=torch.int64, device=device)
        self.col = torch.zeros(max(1, capacity), dtype=torch.int32, device=device)
        self.shift = torch.zeros(max(1, capacity) * 3, dtype=torch.int8, device=device)
        self.rev = torch.zeros(max(1, capacity), dtype=torch.int32, device=device)
        self.n_edges = torch.zeros(1, dtype=torch.int64, device=device)
        self.status = torch.zeros(1, dtype=torch.int32, device=device)

    def struct(self) -> _abi.Nlist:
        n = _abi.Nlist()
        n.capacity = self.capacity
        n.row_ptr = _ptr(self.row_ptr)
        n.col = _ptr(self.col)
        n.shift = _ptr(self.shift)
        n.rev = _ptr(self.rev)
        n.n_edges = _ptr(self.n_edges)
        n.status = _ptr(self.status)
        return n


class Workspace:
    """Planned and allocated device scratch (afm_workspace_plan)."""

    def __init__(self, model: Optional[Model], n_atoms: int, n_struct: int, capacity: int,
                 max_bytes: int = 0, second_order: bool = False, device=None):
        lib = load()
        w = _abi.Workspace()
        check("afm_workspace_plan",
              lib.afm_workspace_plan(model.handle if model else None, n_atoms, n_struct, capacity,
                                     max_bytes, int(second_order), C.byref(w)))
        dev = model.device if model else device
        self.buf = torch.empty(int(w.bytes) + 256, dtype=torch.uint8, device=dev)
        base = self.buf.data_ptr()
        w.ptr = (base + 255) & ~255
        self.ws = w

    @property
    def n_chunks(self) -> int:
        return int(self.ws.n_chunks)


class Calculator:
    """Binds a model, a device system, a neighbour list and a workspace."""

    def __init__(self, model: Model, sysd: DeviceSystem, r_list: Optional[float] = None,
                 capacity: Optional[int] = None, max_bytes: int = 0, second_order: bool = False):
        self.model = model
        self.sysd = sysd
        self.r_list = float(model.hp["r_cut"] if r_list is None else r_list)
        dev = model.device
        N, B = sysd.n_atoms, sysd.n_struct
        if capacity is None:
            capacity = self._estimate_capacity()
        self.nl = NeighborList(N, capacity, dev)
        self.ws = Workspace(model, N, B, capacity, max_bytes, second_order)
        self.lib = load()
        # generation counters of the workspace's per-edge state and of the
        # neighbour list (see energy_and_forces), and the positions the list
        # was last built from (None = sysd.pos)
        self.state_gen = 0
        self.nl_gen = 0
        self.nl_pos = None

    def _estimate_capacity(self) -> int:
        # one build with a probe list to learn the edge count (host sync)
        N, B = self.sysd.n_atoms, self.sysd.n_struct
        probe = NeighborList(N, 0, self.model.device)
        ws = Workspace(None, N, B, 0, device=self.model.device)
        with torch.cuda.device(self.model.device):
            check("afm_build_neighbors",
                  load().afm_build_neighbors(C.byref(self.sysd.struct()), self.r_list,
                                             C.byref(probe.struct()), C.byref(ws.ws),
                                             _stream_ptr(self.model.device)))
            n = int(probe.n_edges.item())
        return max(16, int(n * 1.1) + 64)

    def build_neighbors(self, pos: Optional[torch.Tensor] = None):
        with torch.cuda.device(self.model.device):
            check("afm_build_neighbors",
                  self.lib.afm_build_neighbors(C.byref(self.sysd.struct(pos)), self.r_list,
                                               C.byref(self.nl.struct()), C.byref(self.ws.ws),
                                               _stream_ptr(self.model.device)))
        self.nl_gen += 1
        self.nl_pos = None if pos is None else pos.detach()
        self.state_gen += 1       # the list build uses the workspace's scratch

    def status(self) -> int:
        return int(self.nl.status.item())

    def tune_edge_tile(self, cache_path: Optional[str] = None) -> Dict:
        """Pick the model's edge-tile shape by timing this workload (see
        afm_tune_edge_tile); the list must be built.  Returns the chosen
        shape, the per-shape times (ms) and whether the cache answered."""
        e, w, hit = C.c_int32(), C.c_int32(), C.c_int32()
        ms = (C.c_double * len(_abi.TILE_SHAPES))()
        with torch.cuda.device(self.model.device):
            check("afm_tune_edge_tile",
                  self.lib.afm_tune_edge_tile(self.model.handle, C.byref(self.sysd.struct()),
                                              C.byref(self.nl.struct()), C.byref(self.ws.ws),
                                              cache_path.encode() if cache_path else None, C.byref(e), C.byref(w),
                                              ms, C.byref(hit), _stream_ptr(self.model.device)))
        self.state_gen += 1
        return dict(tile=(int(e.value), int(w.value)), from_cache=bool(hit.value),
                    ms={f"{a}x{b}": float(ms[k]) for k, (a, b) in enumerate(_abi.TILE_SHAPES)})

    def model_n_params(self) -> int:
        return int(sum(b["size"] for b in param_layout(self.model.hp)))

    def forces_backward(self, grad_e_struct=None, grad_forces=None, grad_virial=None, want_pos: bool = False):
        """Weight gradient of J = sum gE E + sum gF . F + sum gW : W (needs
        second_order=True); with want_pos also dJ/dr (float64 [N, 3]),
        returned as (grad_weights, grad_pos)."""
        return _forces_backward(self, grad_e_struct, grad_forces, grad_virial=grad_virial, want_pos=want_pos)

    def _outs(self, forces: bool):
        dev = self.model.device
        N, B = self.sysd.n_atoms, self.sysd.n_struct
        e_atom = torch.empty(N, dtype=torch.float64, device=dev)
        e_struct = torch.empty(B, dtype=torch.float64, device=dev)
        F = torch.empty(N, 3, dtype=torch.float64, device=dev) if forces else None
        W = torch.empty(B, 3, 3, dtype=torch.float64, device=dev) if forces else None
        return e_atom, e_struct, F, W

    def energy_forces(self, pos: Optional[torch.Tensor] = None, virial: bool = True) -> Dict:
        e_atom, e_struct, F, W = self._outs(True)
        with torch.cuda.device(self.model.device):
            check("afm_energy_forces",
                  self.lib.afm_energy_forces(self.model.handle, C.byref(self.sysd.struct(pos)),
                                             C.byref(self.nl.struct()), _ptr(e_atom), _ptr(e_struct),
                                             _ptr(F), _ptr(W) if virial else None, C.byref(self.ws.ws),
                                             _stream_ptr(self.model.device)))
        self.state_gen += 1
        return dict(e_atom=e_atom, e_struct=e_struct, forces=F, virial=W if virial else None)

    def energy_forces_noalloc(self, out: Optional[Dict] = None, pos: Optional[torch.Tensor] = None,
                              virial: bool = True) -> Dict:
        """energy_forces through afm_energy_forces_noalloc: the library's
        static device scratch instead of this calculator's workspace.  `out`
        (from a previous call) supplies the output tensors, so that a call
        allocates nothing."""
        if out is None:
            e_atom, e_struct, F, W = self._outs(True)
            out = dict(e_atom=e_atom, e_struct=e_struct, forces=F, virial=W if virial else None)
        with torch.cuda.device(self.model.device):
            check("afm_energy_forces_noalloc",
                  self.lib.afm_energy_forces_noalloc(self.model.handle, C.byref(self.sysd.struct(pos)),
                                                     C.byref(self.nl.struct()), _ptr(out["e_atom"]),
                                                     _ptr(out["e_struct"]), _ptr(out["forces"]),
                                                     _ptr(out["virial"]), _stream_ptr(self.model.device)))
        return out

    def forward_energy(self, pos: Optional[torch.Tensor] = None):
        e_atom, e_struct, _, _ = self._outs(False)
        with torch.cuda.device(self.model.device):
            check("afm_forward_energy",
                  self.lib.afm_forward_energy(self.model.handle, C.byref(self.sysd.struct(pos)),
                                              C.byref(self.nl.struct()), _ptr(e_atom), _ptr(e_struct),
                                              C.byref(self.ws.ws), _stream_ptr(self.model.device)))
        self.state_gen += 1
        return e_atom, e_struct

    def backward_forces(self, grad_e_struct: Optional[torch.Tensor] = None,
                        pos: Optional[torch.Tensor] = None, virial: bool = False):
        """Forces (and virials) of the last forward_energy call, which must be
        the calculator's last call (afm_backward_forces reads its state)."""
        _, _, F, W = self._outs(True)
        g = None if grad_e_struct is None else grad_e_struct.to(torch.float64).contiguous()
        with torch.cuda.device(self.model.device):
            check("afm_backward_forces",
                  self.lib.afm_backward_forces(self.model.handle, C.byref(self.sysd.struct(pos)),
                                               C.byref(self.nl.struct()), _ptr(g), _ptr(F),
                                               _ptr(W) if virial else None, C.byref(self.ws.ws),
                                               _stream_ptr(self.model.device)))
        self.state_gen += 1
        return F, (W if virial else None)


def _forces_backward(calc: "Calculator", grad_e_struct: Optional[torch.Tensor],
                     grad_forces: Optional[torch.Tensor], pos: Optional[torch.Tensor] = None,
                     grad_virial: Optional[torch.Tensor] = None, want_pos: bool = False):
    """d/dtheta [sum gE E + sum gF . F + sum gW : W] (float32, flat weight
    layout); with want_pos also its position gradient (float64 [N, 3])."""
    dev = calc.model.device
    g = torch.empty(calc.model_n_params(), dtype=torch.float32, device=dev)
    gp = torch.empty(calc.sysd.n_atoms, 3, dtype=torch.float64, device=dev) if want_pos else None
    gE = None if grad_e_struct is None else grad_e_struct.to(torch.float64).contiguous()
    gF = None if grad_forces is None else grad_forces.to(torch.float64).contiguous()
    gW = None if grad_virial is None else grad_virial.to(torch.float64).contiguous()
    with torch.cuda.device(dev):
        check("afm_backward_forces_backward",
              calc.lib.afm_backward_forces_backward(calc.model.handle, C.byref(calc.sysd.struct(pos)),
                                                    C.byref(calc.nl.struct()), _ptr(gE), _ptr(gF), _ptr(gW),
                                                    _ptr(g), _ptr(gp), C.byref(calc.ws.ws), _stream_ptr(dev)))
    calc.state_gen += 1
    return (g, gp) if want_pos else g


class _ForceMatchFn(torch.autograd.Function):
    """(E_s, F, W_s) as functions of a proxy weight tensor: the backward
    returns the weight gradient of sum gE E + sum gF . F + sum gW : W from the
    library's second-order entry point (the weights themselves live in the
    model)."""

    @staticmethod
    def forward(ctx, theta, calc):
        out = calc.energy_forces(virial=True)
        ctx.calc = calc
        ctx.theta_meta = (theta.device, theta.dtype)
        ctx.set_materialize_grads(False)     # unused outputs arrive as None
        return out["e_struct"], out["forces"], out["virial"]

    @staticmethod
    def backward(ctx, gE, gF, gW):
        g = _forces_backward(ctx.calc, gE, gF, grad_virial=gW)
        dev, dt = ctx.theta_meta
        return g.to(device=dev, dtype=dt), None


def energy_forces_for_training(calc: "Calculator", theta: torch.Tensor, virial: bool = False):
    """E_s and F (and the virials W_s if `virial`) whose gradients flow to
    `theta` (a float64 tensor standing for the model's weights; requires a
    calculator with second_order=True)."""
    E, F, W = _ForceMatchFn.apply(theta, calc)
    return (E, F, W) if virial else (E, F)


class Adam:
    """Adam on the model's flat weight vector: step(grad) applies
    afm_adam_step to a device float64 copy of the weights and repacks the
    model with afm_model_set_weights."""

    def __init__(self, model: Model, weights: np.ndarray, lr: float = 1e-3, betas=(0.9, 0.999),
                 eps: float = 1e-8):
        dev = model.device
        self.model = model
        self.theta = torch.as_tensor(np.ascontiguousarray(weights, np.float64), device=dev).clone()
        self.m1 = torch.zeros_like(self.theta)
        self.m2 = torch.zeros_like(self.theta)
        self.lr, self.betas, self.eps, self.t = float(lr), betas, float(eps), 0

    def step(self, grad: torch.Tensor):
        g = grad.to(device=self.theta.device, dtype=torch.float32).contiguous()
        self.t += 1
        dev = self.model.device
        with torch.cuda.device(dev):
            check("afm_adam_step", load().afm_adam_step(
                _ptr(self.theta), _ptr(g), _ptr(self.m1), _ptr(self.m2), self.theta.numel(), self.lr,
                float(self.betas[0]), float(self.betas[1]), self.eps, self.t, _stream_ptr(dev)))
        self.model.set_weights(self.theta.cpu().numpy())


class _EnergyFn(torch.autograd.Function):
    """E_s(pos); its backward returns -forces weighted by the upstream grad.

    afm_backward_forces reads the per-edge state afm_forward_energy left in
    the workspace (and the calculator's neighbour list).  If the calculator
    ran anything else in between -- another forward, a list rebuild -- the
    backward first rebuilds the list (if it was rebuilt) and re-runs the
    forward at the saved positions, so each E_s gets its own forces."""

    @staticmethod
    def forward(ctx, pos, calc):
        if calc.nl_gen == 0:
            raise RuntimeError("build the neighbour list (calc.build_neighbors) before energy_and_forces")
        p = pos.detach()
        e_atom, e_struct = calc.forward_energy(p)
        ctx.calc = calc
        ctx.gens = (calc.state_gen, calc.nl_gen, calc.nl_pos)
        ctx.save_for_backward(pos)
        return e_struct

    @staticmethod
    def backward(ctx, grad_e):
        (pos,) = ctx.saved_tensors
        calc = ctx.calc
        p = pos.detach()
        state_gen, nl_gen, nl_pos = ctx.gens
        if calc.nl_gen != nl_gen:
            calc.build_neighbors(nl_pos)
        if calc.state_gen != state_gen:
            calc.forward_energy(p)
        F, _ = calc.backward_forces(grad_e.contiguous(), pos=p)
        return -F, None


class EvalGraph:
    """One evaluation step of a calculator -- the edge-list build (optional)
    and afm_energy_forces -- captured once into a hipGraph on the current
    stream and replayed: the launches of every stage for the whole batch go
    out as one graph launch.  The outputs live in fixed tensors (`out`),
    overwritten by each replay; positions are read from calc.sysd.pos at
    replay time (update it in place)."""

    def __init__(self, calc: Calculator, rebuild: bool = True, virial: bool = True):
        self.calc = calc
        dev = calc.model.device
        self.rebuild = rebuild
        e_atom, e_struct, F, W = calc._outs(True)
        self.out = dict(e_atom=e_atom, e_struct=e_struct, forces=F, virial=W if virial else None)
        self._nl = calc.nl.struct()
        self._sys = calc.sysd.struct()
        # one eager step first (same launches, so nothing is set up during
        # the capture), then the capture
        self._step(_stream_ptr(dev))
        torch.cuda.synchronize(dev)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self._step(_stream_ptr(dev))
        torch.cuda.synchronize(dev)

    def _step(self, stream):
        lib, calc, o = load(), self.calc, self.out
        with torch.cuda.device(calc.model.device):
            if self.rebuild:
                check("afm_build_neighbors",
                      lib.afm_build_neighbors(C.byref(self._sys), calc.r_list, C.byref(self._nl),
                                              C.byref(calc.ws.ws), stream))
            check("afm_energy_forces",
                  lib.afm_energy_forces(calc.model.handle, C.byref(self._sys), C.byref(self._nl),
                                        _ptr(o["e_atom"]), _ptr(o["e_struct"]), _ptr(o["forces"]),
                                        _ptr(o["virial"]), C.byref(calc.ws.ws), stream))

    def replay(self) -> Dict:
        self.graph.replay()
        self.calc.state_gen += 1
        if self.rebuild:
            self.calc.nl_gen += 1
            self.calc.nl_pos = None
        return self.out


def energy_and_forces(calc: Calculator, pos: torch.Tensor) -> torch.Tensor:
    """Differentiable E_s(pos) (forces = -dE/dpos through autograd)."""
    return _EnergyFn.apply(pos, calc)


class MD:
    """Velocity-Verlet driver over afm_md_step: NVE, or NVT with a Nose-Hoover
    thermostat when t_target_K > 0 (period tau_fs, n_dof degrees of freedom,
    3 N by default).  Positions are updated in place in calc.sysd.pos; calc
    must have been built with r_list = r_cut + skin.  With use_graph the steps
    run on a private stream and are replayed from a captured hipGraph after
    the first call of each phase."""

    def __init__(self, calc: Calculator, masses_by_species, v0, dt_fs: float = 0.5, skin: float = 0.5,
                 rebuild_every: int = 10, use_graph: bool = False, t_target_K: float = 0.0,
                 tau_fs: float = 100.0, n_dof: int = 0, xi0: float = 0.0, eta0: float = 0.0):
        dev = calc.model.device
        self.calc = calc
        self.stream = torch.cuda.Stream(dev) if use_graph else None
        N, B = calc.sysd.n_atoms, calc.sysd.n_struct
        self.mass = torch.as_tensor(np.asarray(masses_by_species, np.float64), device=dev)
        self.vel = torch.as_tensor(np.ascontiguousarray(v0, np.float64), device=dev).reshape(N, 3).contiguous()
        self.e_atom = torch.zeros(N, dtype=torch.float64, device=dev)
        self.e_struct = torch.zeros(B, dtype=torch.float64, device=dev)
        calc.build_neighbors()
        out = calc.energy_forces(virial=False)
        self.forces = out["forces"]
        st = _abi.MdState()
        st.pos = _ptr(calc.sysd.pos)
        st.vel = _ptr(self.vel)
        st.forces = _ptr(self.forces)
        st.mass_by_species = _ptr(self.mass)
        st.dt_fs = float(dt_fs)
        st.skin = float(skin)
        st.rebuild_every = int(rebuild_every)
        st.use_graph = int(use_graph)
        st.step = 0
        st.e_atom = _ptr(self.e_atom)
        st.e_struct = _ptr(self.e_struct)
        # thermostat state (xi, eta, two scratch words), carried across calls
        self.nh = torch.tensor([xi0, eta0, 1.0, 0.0], dtype=torch.float64, device=dev)
        st.t_target_K = float(t_target_K)
        st.tau_fs = float(tau_fs)
        st.n_dof = int(n_dof)
        st.nh = _ptr(self.nh)
        st.thermostat_log = None
        self.state = st
        self._logs = {}
        self._tlogs = {}
        self.thermostat_log = None

    def run(self, n_steps: int) -> torch.Tensor:
        """Advance n_steps; returns the [n_steps, 2] (kinetic, potential) log
        (NVT: the thermostat energies of the steps go to self.thermostat_log)."""
        dev = self.calc.model.device
        log = self._logs.get(n_steps)
        if log is None:
            log = torch.zeros(n_steps, 2, dtype=torch.float64, device=dev)
            self._logs[n_steps] = log
        self.state.energy_log = _ptr(log)
        if self.state.t_target_K > 0:
            tlog = self._tlogs.get(n_steps)
            if tlog is None:
                tlog = torch.zeros(n_steps, dtype=torch.float64, device=dev)
                self._tlogs[n_steps] = tlog
            self.state.thermostat_log = _ptr(tlog)
        if self.stream is not None:
            self.stream.wait_stream(torch.cuda.current_stream(dev))
            with torch.cuda.stream(self.stream):
                check("afm_md_step", load().afm_md_step(
                    self.calc.model.handle, C.byref(self.calc.sysd.struct()), C.byref(self.calc.nl.struct()),
                    C.byref(self.state), n_steps, C.byref(self.calc.ws.ws), C.c_void_p(self.stream.cuda_stream)))
            torch.cuda.current_stream(dev).wait_stream(self.stream)
        else:
            with torch.cuda.device(dev):
                check("afm_md_step", load().afm_md_step(
                    self.calc.model.handle, C.byref(self.calc.sysd.struct()), C.byref(self.calc.nl.struct()),
                    C.byref(self.state), n_steps, C.byref(self.calc.ws.ws), _stream_ptr(dev)))
        self.calc.state_gen += 1
        self.calc.nl_gen += 1
        self.calc.nl_pos = None
        if self.state.t_target_K > 0:
            # thermostat energy Q xi^2/2 + g kB T eta per step (eV)
            self.thermostat_log = self._tlogs[n_steps].clone()
        return log.clone()
