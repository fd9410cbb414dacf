"""FP64 CPU oracle for deep-potential energy, forces and virial -- TEST INFRASTRUCTURE ONLY.

This package is the slow, plain reference that the HIP library is checked
against.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg
of ``bench.py`` may import it; the library never does, and the oracle shares
no code with the library (only the seeded inputs from :mod:`synth` and the
model-file format, which each side parses with its own reader).

What it computes, in the paper's terms (Section II: an embedding net over
each atom's neighbours with type information, self-attention layers that
update that representation residually, a fitting net that gives each atom's
energy, E the sum over atoms; Section II, forces are minus the gradient of
the potential; neighbour lists within a cutoff, Section II and IV):

* :mod:`oracle.neighbors` -- brute-force O(N^2) neighbour lists under an
  exact FP64 rule, and an independent cell-list search that must equal it;
* :mod:`oracle.dp` -- the model forward, its reverse-mode gradient written by
  hand, forces by gather, virial, per-atom evaluation of a subset, and models
  with several fitting heads on one descriptor;
* :mod:`oracle.gnn` -- the GNN-variant descriptor (message passing over edges and
  angles, three layers) with its hand-written gradient;
* :mod:`oracle.repformer` -- a repformer-style model (pair and node features, gated
  self-attention over the neighbours' pair features, neighbour-to-neighbour message
  passing, three layers) with its hand-written gradient;
* :mod:`oracle.nve` -- a velocity-Verlet driver for the energy-drift check.

The paper prints no model equations; the functional form follows the reading
stated in oracle/dp.py (quintic switch, switch-weighted gated softmax,
residual LayerNorm update, 1/sel descriptor normalisation).  Every function
here is pinned by tests under ``tests/`` against closed forms, brute force,
special cases and finite differences; the agreement with the paper's trained
DPA models themselves is parity unpinned (no weights, no equations).
"""
from .model_file import load_model  # noqa: F401
from .neighbors import neighbor_list_bruteforce, neighbor_list_cells  # noqa: F401
from .dp import (  # noqa: F401
    switch, atom_energy_and_grad, evaluate, evaluate_subset, forces_from_pairs, head_view, evaluate_heads,
)
