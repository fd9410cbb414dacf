"""MI355X (gfx950) deep-potential energy, force and virial library.

The computation lives in ``libdp.so`` (hand-written HIP kernels behind a C ABI,
include/dp.h); this package only marshals arguments to it.
"""
from ._lib import DP_BF16, DP_FP32, DPError, load  # noqa: F401
from .api import GnnModel, Model, RepModel, Server, energy  # noqa: F401

__all__ = ["Model", "GnnModel", "RepModel", "Server", "energy", "DPError", "DP_FP32", "DP_BF16", "load"]
