"""Shared helpers of the GPU tests: run the HIP path through the C ABI and
compare with the oracle."""

import numpy as np

import synth


def weights_for(hp, seed):
    from oracle import model as M
    return synth.draw_weights(M.param_layout(M.HParams.from_dict(hp)), seed)


def gpu_run(hp, weights, s, precision="fp32", r_list=None, max_bytes=0, capacity=None):
    import torch
    import paper_2502_06073_amd as afm
    model = afm.Model(hp, weights, precision=precision)
    sysd = afm.DeviceSystem.from_synth(s)
    calc = afm.Calculator(model, sysd, r_list=r_list, max_bytes=max_bytes, capacity=capacity)
    calc.build_neighbors()
    out = calc.energy_forces()
    torch.cuda.synchronize()
    res = {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}
    res["status"] = calc.status()
    res["n_chunks"] = calc.ws.n_chunks
    res["calc"] = calc
    return res


def gpu_nlist(calc):
    n = int(calc.nl.n_edges.item())
    return dict(row_ptr=calc.nl.row_ptr.cpu().numpy(),
                j=calc.nl.col[:n].cpu().numpy().astype(np.int64),
                n=calc.nl.shift[:3 * n].cpu().numpy().astype(np.int64).reshape(-1, 3),
                rev=calc.nl.rev[:n].cpu().numpy().astype(np.int64))


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (den if den > 0 else 1.0))


def mu_of(hp, weights, s):
    from oracle import model as M
    lay = M.param_layout(M.HParams.from_dict(hp))
    off = sum(b["size"] for b in lay[:-1])
    return weights[off:off + hp["n_species"]][s.species]


def parity_report(hp, weights, s, gpu, ref):
    """Errors of the R15 kind: relative norms of (E_i - mu), F, W and
    |dE_s| / sum |E_i - mu|; plus the absolute per-atom and force-RMS
    figures used for the BF16 path."""
    mu = mu_of(hp, weights, s)
    ea_g = gpu["e_atom"] - mu
    ea_r = ref["e_atom"] - mu
    n_s = np.diff(s.seg)
    out = dict(
        e_atom=rel(ea_g, ea_r),
        e_struct=float(np.max(np.abs(gpu["e_struct"] - ref["e_struct"])) / max(np.sum(np.abs(ea_r)), 1e-30)),
        forces=rel(gpu["forces"], ref["forces"]),
        virial=rel(gpu["virial"], ref["virial"]),
        e_per_atom_abs=float(np.max(np.abs(gpu["e_struct"] - ref["e_struct"]) / n_s)),
        force_rms_abs=float(np.sqrt(np.mean((gpu["forces"] - ref["forces"]) ** 2))),
    )
    return out


def weights_nonunit(hp, seed):
    """Seeded weights with the blocks whose default is all ones drawn away
    from 1: every path-mixing weight alpha ~ +-U(0.4, 1.6) and every species
    energy scale sigma_Z ~ U(0.5, 1.5) (the other blocks as weights_for)."""
    from oracle import model as M
    lay = M.param_layout(M.HParams.from_dict(hp))
    w = synth.draw_weights(lay, seed)
    rng = np.random.Generator(np.random.PCG64(seed + 7919))
    off = 0
    for b in lay:
        n = b["size"]
        if b["name"].endswith(".alpha"):
            w[off:off + n] = rng.uniform(0.4, 1.6, n) * rng.choice([-1.0, 1.0], n)
        elif b["name"] == "species.scale":
            w[off:off + n] = rng.uniform(0.5, 1.5, n)
        off += n
    return w
