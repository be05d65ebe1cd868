"""Throughput of the energy+force hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config B]

Workload (default): the 13,824-atom periodic system (24^3 simple-cubic
lattice, spacing 2.2 A, +-0.25 A uniform jitter, 4 species drawn uniformly,
cutoff 5.5 A, l_max = 2, 2 layers, latent width 256, 3-layer MLPs, 8 Bessel
functions), seeded synthetic positions and N(0, 1/fan_in) weights.  One
step = build the edge list + energies + forces + virial (every step of the
path), with inputs resident in HBM.  The BF16-MFMA path is timed as the
headline value; the plain-FP32 path is timed beside it for the speedup.

Prints one JSON line with, besides the contract fields, a "roofline" entry
for the dominant kernel (algorithmic FLOPs per launch / its average HIP-event
duration during the timed steps) and a "cpu_baseline" entry (the FP64 oracle
on a bounded sample of central atoms, on the host's cores), plus the force
RMS error of both GPU paths against the FP64 oracle on sampled atoms.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_BF16 = 2.5e15      # dense BF16 MFMA, FLOP/s
PEAK_FP32 = 157.3e12    # FP32 vector, FLOP/s


def mlp_macs_per_edge(hp):
    """Multiply-accumulates per edge of each GEMM stage (algorithmic work of
    the MLP kernels; the forward of a stage and its input-gradient adjoint
    do the same number)."""
    from oracle import model as M  # noqa: F401  (path enumeration only in the oracle)
    w, c, lm = hp["latent"], hp["channels"], hp["l_max"]
    env = (lm + 1) * c
    tb = hp["twobody"]
    S, nb = hp["n_species"], hp["n_bessel"]
    n0e = 3 if lm == 2 else lm + 1
    tb_macs = nb * tb[0] + sum(tb[k - 1] * tb[k] for k in range(1, len(tb))) + w * env
    lat = (w + n0e * c) * w + (hp["latent_depth"] - 1) * w * w
    out = {"twobody_fwd": tb_macs, "twobody_bwd": tb_macs}
    NL = hp["n_layers"]
    for L in range(1, NL + 1):
        extra_f = w * env if L < NL else w
        extra_b = w * env if L < NL else 0
        out[f"latent_fwd{L}"] = lat + extra_f
        out[f"latent_bwd{L}"] = lat + extra_b
    return out


def setup(config, precision):
    import torch
    import synth
    import paper_2502_06073_amd as afm
    hp = synth.load_hparams(config)
    s = synth.SYSTEMS[config]()
    w = synth.draw_weights(afm.param_layout(hp), synth.WEIGHT_SEEDS[config])
    model = afm.Model(hp, w, precision=precision)
    sysd = afm.DeviceSystem.from_synth(s)
    calc = afm.Calculator(model, sysd, r_list=hp.get("r_list", hp["r_cut"]))
    calc.build_neighbors()
    torch.cuda.synchronize()
    return hp, s, w, calc


def time_steps(calc, steps, warmup, trace=False):
    import torch
    import paper_2502_06073_amd as afm
    for _ in range(warmup):
        calc.build_neighbors()
        calc.energy_forces()
    torch.cuda.synchronize()
    if trace:
        afm.trace_enable(True)
    t0 = time.perf_counter()
    out = None
    for _ in range(steps):
        calc.build_neighbors()
        out = calc.energy_forces()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    stats = None
    if trace:
        stats = afm.trace_read()
        afm.trace_enable(False)
    return dt, out, stats


def cpu_baseline(hp, s, w, budget_s=15.0):
    """The FP64 oracle, as it stands, on a bounded sample of central atoms
    (E_i and dE/d delta of their edges: the per-atom work of one step)."""
    import torch
    import synth
    from oracle import model as M
    rows = synth.subset_rows(s.n_atoms, 32, 7)
    t0 = time.perf_counter()
    M.rows_energy_grad(hp, w, s, rows, r_list=hp.get("r_list", hp["r_cut"]))
    t1 = time.perf_counter() - t0
    k = int(min(s.n_atoms, max(32, 32 * budget_s / max(t1, 1e-3))))
    rows = synth.subset_rows(s.n_atoms, k, 8)
    t0 = time.perf_counter()
    M.rows_energy_grad(hp, w, s, rows, r_list=hp.get("r_list", hp["r_cut"]))
    t = time.perf_counter() - t0
    return dict(value=k / t, unit="atom-steps/s", cores=int(torch.get_num_threads()), kind="oracle",
                sample=f"{k} seeded central atoms (E_i and dE/d delta_e of their rows), FP64, "
                       f"{t:.1f} s; os.cpu_count()={os.cpu_count()}")


def force_errors(hp, s, w, outs, n_atoms=8):
    import synth
    from oracle import model as M
    atoms = synth.subset_rows(s.n_atoms, n_atoms, 101)
    ref = M.forces_subset(hp, w, s, atoms, r_list=hp.get("r_list", hp["r_cut"]))
    res = {}
    for name, out in outs.items():
        F = out["forces"].cpu().numpy()[atoms]
        E = out["e_atom"].cpu().numpy()[atoms]
        res[name] = dict(force_rms_err=float(np.sqrt(np.mean((F - ref["forces"]) ** 2))),
                         force_rel_err=float(np.linalg.norm(F - ref["forces"]) / np.linalg.norm(ref["forces"])),
                         e_atom_max_abs_err=float(np.abs(E - ref["e_atom"]).max()))
    res["sample_atoms"] = int(n_atoms)
    res["ref_force_rms"] = float(np.sqrt(np.mean(ref["forces"] ** 2)))
    return res


def load_traffic(kernel_stage):
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            d = json.load(f)
        return d.get(kernel_stage)
    except Exception:
        return None


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="B")
    ap.add_argument("--fp32-steps", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    a = ap.parse_args(argv)
    if a.gpus != 1:
        print(f"bench.py measures one GPU only (the path runs on a single MI355X); "
              f"--gpus {a.gpus} is not supported", file=sys.stderr)
        return 2
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    print(f"[bench] config {a.config}: setting up bf16", file=sys.stderr, flush=True)
    hp, s, w, calc = setup(a.config, "bf16")
    n_edges = int(calc.nl.n_edges.item())
    dt, out_bf16, stats = time_steps(calc, a.steps, a.warmup, trace=True)
    ms = dt / a.steps * 1e3
    value = s.n_atoms * a.steps / dt
    print(f"[bench] bf16: {ms:.3f} ms/step, {value:.4g} atom-steps/s", file=sys.stderr, flush=True)
    macs = mlp_macs_per_edge(hp)
    # dominant kernel: the stage with the largest GPU time
    dom = max(stats.items(), key=lambda kv: kv[1]["total_ms"])
    dom_name, dom_st = dom
    avg_ms = dom_st["total_ms"] / dom_st["launches"]
    roof = None
    if dom_name in macs:
        flops = 2.0 * macs[dom_name] * n_edges
        ach = flops / (avg_ms * 1e-3)
        roof = dict(bound="mfma", kernel=dom_name, achieved=ach / 1e12, peak=PEAK_BF16 / 1e12,
                    unit="TFLOP/s", frac=ach / PEAK_BF16, traffic=load_traffic(dom_name),
                    flops_per_launch=flops, avg_ms=avg_ms)
    # whole-step MLP FLOP rate (all MFMA stages)
    mlp_flops = sum(2.0 * v * n_edges for v in macs.values())
    stage_ms = {k: round(v["total_ms"] / v["launches"], 4) for k, v in stats.items()}
    out = dict(metric="atom-steps/s energy+forces, BF16-MFMA vs FP32 plain; force RMS err vs FP64",
               value=value, unit="atom-steps/s", n_gpus=1, steps=a.steps, warmup=a.warmup, ms_per_step=ms,
               higher_is_better=True, scaling="weak", vs_baseline=None, dtype="bf16",
               data="synthetic (seeded jittered lattice, N(0,1/fan_in) weights)",
               config=dict(workload=f"{s.n_atoms}-atom periodic jittered SC lattice (24^3, a=2.2 A), 4 species, "
                                    f"r_c 5.5 A, l_max 2, 2 layers, latent 256, 3-layer MLPs, energy+forces+virial "
                                    f"incl. edge-list build" if a.config == "B" else f"config {a.config}",
                           n_atoms=s.n_atoms, n_edges=n_edges, parallelism="single GPU"),
               roofline=roof, stage_ms=stage_ms,
               mlp_tflops_per_step=mlp_flops / (ms * 1e-3) / 1e12)
    outs = {"bf16": out_bf16}
    if not a.no_fp32:
        print("[bench] timing fp32 plain", file=sys.stderr, flush=True)
        _, _, _, calc32 = setup(a.config, "fp32")
        dt32, out32, st32 = time_steps(calc32, a.fp32_steps, 1, trace=True)
        v32 = s.n_atoms * a.fp32_steps / dt32
        out["fp32_plain"] = dict(value=v32, ms_per_step=dt32 / a.fp32_steps * 1e3,
                                 stage_ms={k: round(v["total_ms"] / v["launches"], 4) for k, v in st32.items()})
        out["speedup_bf16_vs_fp32"] = value / v32
        outs["fp32"] = out32
        print(f"[bench] fp32: {dt32 / a.fp32_steps * 1e3:.2f} ms/step", file=sys.stderr, flush=True)
    if not a.no_cpu_baseline:
        print("[bench] oracle CPU baseline and FP64 errors", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(hp, s, w)
        out["error_vs_fp64"] = force_errors(hp, s, w, outs)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
