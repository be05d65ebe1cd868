"""FP64 CPU oracle for the strictly-local equivariant edge potential.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or
link this package: only the test-suite, the smoke check and the CPU-baseline
leg of the benchmark use it.  It shares no code with the HIP library; the
only common inputs come from the seeded generators in ``synth``.

The method (Allegro, the architecture the paper trains as Allegro-FM; see the
paper's Methodology / Model Training section and Table 1) is written out here
plainly in float64, step by step, in the paper's vocabulary:

* ``neighbors``  directed edge list within the cutoff, all periodic images,
  canonical order (the "strictly-local" neighbourhoods of the Abstract).
* ``so3``        real spherical harmonics and real Clebsch-Gordan tensors
  derived numerically from their defining invariance.
* ``model``      two-body latent MLP, environment embeddings, channelwise
  tensor products with the summed neighbour environment, latent MLPs, edge
  energies, per-atom and total energies; forces and virial by autograd;
  training loss and its weight gradient by double backward.
* ``md``         velocity-Verlet NVE dynamics.

Readings of points the paper leaves open are listed in each module header.
Functions without an external pin are marked "parity unpinned".
"""

import importlib as _il

__all__ = ["neighbors", "so3", "model", "md"]


def __getattr__(name):
    if name in __all__:
        return _il.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
