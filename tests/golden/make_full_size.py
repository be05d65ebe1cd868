"""Write tests/golden/full_size_energies.json: FP64 oracle energies of the
full-size seeded workloads, for the GPU parity tests that run those
workloads whole (the oracle takes minutes on them, the tests seconds).

* B: the 13,824-atom periodic lattice (E_s, and E_i of 512 seeded atoms);
* C: the 64 open clusters (E_s of every structure);
* D: the 512 uneven structures (E_s of every structure).

Seeded structures and weights of each workload as the benchmark uses them
(synth.SYSTEMS, synth.WEIGHT_SEEDS, tests/golden/hparams.json); energies
only (no forces), computed by the oracle alone.

Run:  python tests/golden/make_full_size.py
"""

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import model  # noqa: E402

ATOM_SAMPLE_SEED = 307


def main():
    out = {}
    for name in "BCD":
        t0 = time.time()
        hp = synth.load_hparams(name)
        s = synth.SYSTEMS[name]()
        w = synth.draw_weights(model.param_layout(model.HParams.from_dict(hp)), synth.WEIGHT_SEEDS[name])
        r = model.energy_forces(model.HParams.from_dict(hp), w, s, want_forces=False)
        rec = dict(n_atoms=int(s.n_atoms), n_struct=int(s.n_struct),
                   n_edges=int(r["nl"]["i"].shape[0]),
                   e_struct=[float(v) for v in r["e_struct"]])
        if name == "B":
            rows = synth.subset_rows(s.n_atoms, 512, ATOM_SAMPLE_SEED)
            rec["atom_sample_seed"] = ATOM_SAMPLE_SEED
            rec["e_atom_rows"] = [int(v) for v in rows]
            rec["e_atom"] = [float(v) for v in r["e_atom"][rows]]
        out[name] = rec
        print(f"{name}: {s.n_atoms} atoms, {s.n_struct} structures, {rec['n_edges']} edges, "
              f"{time.time() - t0:.1f} s", flush=True)
    with open(os.path.join(HERE, "full_size_energies.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
