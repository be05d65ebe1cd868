"""Write tests/golden/hparams.json: the two derived hyperparameters of each
workload, measured by the FP64 oracle only.

* avg_num_neighbors (the environment-sum normaliser nbar): mean number of
  edges per atom within the model cutoff on the workload's seeded structure,
  rounded to 3 significant figures (all atoms for A-D; a seeded sample of
  20,000 rows for the 1M-atom workload E).
* energy_scale: set so that the per-component force RMS of the seeded
  weights on the seeded structure is 1 eV/A (forces are linear in it),
  rounded to 6 significant figures.  Measured on all atoms for A and C and
  on 64 seeded atoms (exact local forces) for B, D and E.

Run:  python tests/golden/make_hparams.py
"""

import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import model, neighbors  # noqa: E402


def sig(x, n):
    return float(f"{x:.{n}g}")


def main():
    out = {}
    for name in "ABCDE":
        t0 = time.time()
        cfg = dict(synth.CONFIGS[name])
        sysx = synth.SYSTEMS[name]()
        if name == "E":
            rows = synth.subset_rows(sysx.n_atoms, 20000, 77)
            nl = neighbors.build(sysx, cfg["r_cut"], rows=rows)
            deg = nl["i"].shape[0] / rows.shape[0]
        else:
            nl = neighbors.build(sysx, cfg["r_cut"])
            deg = nl["i"].shape[0] / sysx.n_atoms
        nbar = sig(deg, 3)
        hp = model.HParams.from_dict(cfg)
        hp.avg_num_neighbors = nbar
        hp.energy_scale = 1.0
        W = synth.draw_weights(model.param_layout(hp), synth.WEIGHT_SEEDS[name])
        if name in "AC":
            F = model.energy_forces(hp, W, sysx, nl=nl)["forces"]
            how = "all atoms"
        else:
            atoms = synth.subset_rows(sysx.n_atoms, 64, 78)
            F = model.forces_subset(hp, W, sysx, atoms)["forces"]
            how = "64 seeded atoms (seed 78)"
        rms = math.sqrt(float(np.mean(F * F)))
        out[name] = dict(
            frozen=dict(avg_num_neighbors=nbar,
                        energy_scale=sig(1.0 / rms, 6)),
            notes=dict(mean_degree=deg, force_rms_at_scale_1=rms,
                       force_sample=how, n_atoms=sysx.n_atoms,
                       n_struct=sysx.n_struct))
        print(name, out[name], f"{time.time() - t0:.1f}s", flush=True)
    with open(os.path.join(HERE, "hparams.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
