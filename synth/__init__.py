"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle's checks.

This package draws random numbers and lays out atoms; it holds none of the
deep-potential arithmetic (no switch function, no network, no neighbor test).
Both the FP64 oracle and the HIP library consume what it produces as data:

* :mod:`synth.systems` -- water boxes and water-solvated chains (positions,
  types, periodic cubic box), and the seeded serving request trace;
* :mod:`synth.weights` -- the random-init model parameters and the binary
  model file both sides load.
"""
from .systems import (  # noqa: F401
    TYPE_NAMES, TYPE_INDEX, MASSES, water_box, solvated_chain, config_system,
    serving_trace, request_system,
)
from .weights import ModelSpec, make_params, write_model_file, default_model_file  # noqa: F401
