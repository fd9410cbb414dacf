"""ctypes view of ``libdp.so`` (the C ABI declared in include/dp.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of the shared library.  Loading fails loudly when the library has not
been built (``python -m paper_2602_02234_amd.build``).
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdp.so")

DP_FP32, DP_BF16 = 0, 1
STATUS = {
    0: "DP_OK", 1: "DP_WARN_SEL_OVERFLOW", -1: "DP_ERR_ARG", -2: "DP_ERR_MODEL_FILE", -3: "DP_ERR_TYPE",
    -4: "DP_ERR_BOX", -5: "DP_ERR_OVERLAP", -6: "DP_ERR_NONFINITE", -7: "DP_ERR_OOM", -8: "DP_ERR_TOO_LARGE",
    -9: "DP_ERR_HIP", -10: "DP_ERR_TIMEOUT",
}

_lib = None

_P = C.c_void_p
_I64 = C.c_int64
SIGNATURES = {
    "dp_model_load": (C.c_int, [C.c_char_p, C.c_int, C.c_int, C.POINTER(C.c_void_p)]),
    "dp_model_free": (None, [_P]),
    "dp_check_model_file": (C.c_int, [C.c_char_p, C.c_int, C.c_char_p, C.POINTER(C.c_size_t)]),
    "dp_model_info": (C.c_int, [_P, C.POINTER(C.c_double), C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "dp_compute": (C.c_int, [_P, _I64, _P, _P, _P, _P, _P, _P, _P]),
    "dp_compute_device": (C.c_int, [_P, _I64, _P, _P, _P, _P, _P, _P, _P, _P]),
    "dp_compute_device_noalloc": (C.c_int, [_P, _I64, _P, _P, _P, _P, _P, _P, _P, _P]),
    "dp_compute_owned_device": (C.c_int, [_P, _I64, _I64, _P, _P, _P, _P, _P, _P, _P, _P]),
    "dp_backward_device": (C.c_int, [_P, _P, _P, _P, _P]),
    "dp_debug_neighbors": (C.c_int, [_P, _I64, _P, _P, _P, _P, _P]),
    "dp_debug_pair_grads": (C.c_int, [_P, _I64, _P]),
    "dp_profile_enable": (C.c_int, [_P, C.c_int]),
    "dp_profile_read": (C.c_int, [_P, _P, _P, C.c_int]),
    "dp_compute_batch_device": (C.c_int, [_P, C.c_int, _P, _P, _P, _P, _P, _P, _P, _P]),
    "dp_set_skin": (C.c_int, [_P, C.c_double, C.c_int]),
    "dp_model_heads": (C.c_int, [_P, C.POINTER(C.c_int)]),
    "dp_set_head_weights": (C.c_int, [_P, C.c_int, _P]),
    "dp_head_energies": (C.c_int, [_P, C.c_int, _P]),
    "dp_skin_stats": (C.c_int, [_P, _P, _P]),
    "dp_set_graph": (C.c_int, [_P, C.c_int]),
    "dp_set_chunk": (C.c_int, [_P, _I64]),
    "dp_server_footprint": (C.c_size_t, [_P, _I64]),
    "dp_server_create": (C.c_int, [_P, C.c_size_t, C.c_int, C.POINTER(C.c_void_p)]),
    "dp_submit": (C.c_int, [_P, _I64, _P, _P, _P, C.POINTER(C.c_uint64)]),
    "dp_wait": (C.c_int, [_P, C.c_uint64, C.c_double, _P, _P, _P, _P]),
    "dp_server_stats": (C.c_int, [_P, _P, _P, _P, _P, _P, _P]),
    "dp_server_free": (None, [_P]),
    "dp_nve_run": (C.c_int, [_P, _I64, _P, _P, _P, _P, _P, C.c_double, C.c_int, _P, _P, _P]),
    "dp_gnn_load": (C.c_int, [C.c_char_p, C.c_int, C.c_int, C.POINTER(C.c_void_p)]),
    "dp_gnn_free": (None, [_P]),
    "dp_gnn_info": (C.c_int, [_P, C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_int),
                              C.POINTER(C.c_int)]),
    "dp_gnn_compute_device": (C.c_int, [_P, _I64, _P, _P, _P, _P, _P, _P, _P, _P]),
    "dp_gnn_graph_size": (C.c_int, [_P, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "dp_gnn_profile_enable": (C.c_int, [_P, C.c_int]),
    "dp_gnn_profile_read": (C.c_int, [_P, _P, _P, C.c_int]),
    "dp_rep_load": (C.c_int, [C.c_char_p, C.c_int, C.POINTER(C.c_void_p)]),
    "dp_rep_free": (None, [_P]),
    "dp_rep_compute_device": (C.c_int, [_P, _I64, _P, _P, _P, _P, _P, _P, _P, _P]),
    "dp_rep_edges": (C.c_int, [_P, C.POINTER(C.c_int64)]),
    "dp_rep_profile_enable": (C.c_int, [_P, C.c_int]),
    "dp_rep_profile_read": (C.c_int, [_P, _P, _P, C.c_int]),
    "dp_status_string": (C.c_char_p, [C.c_int]),
    "dp_last_error": (C.c_char_p, []),
}


def load():
    """The loaded library (raises if it is missing: there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2602_02234_amd.build`")
    # PyTorch-ROCm bundles its own HIP runtime.  Loading it first makes this
    # library bind to that same runtime (same soname), so device pointers and
    # streams from torch are valid here; loading ours first would put two HIP
    # runtimes into the process and torch would then find no GPU.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


class DPError(RuntimeError):
    def __init__(self, status: int, where: str):
        lib = load()
        detail = lib.dp_last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS.get(status, status)} ({detail})")
        self.status = status


def check(status: int, where: str) -> int:
    if status < 0:
        raise DPError(status, where)
    return status
