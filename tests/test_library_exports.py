"""The C-ABI library loads and exports every function include/dp.h declares (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "dp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dp_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for f in ("dp_model_load", "dp_model_free", "dp_compute", "dp_compute_device", "dp_backward_device",
              "dp_debug_neighbors", "dp_status_string", "dp_last_error", "dp_model_info"):
        assert f in names


def test_library_exports_every_declared_symbol():
    from paper_2602_02234_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libdp.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(_lib.SIGNATURES) == set(_declared())


def test_status_strings_without_gpu():
    from paper_2602_02234_amd import _lib
    lib = _lib.load()
    assert lib.dp_status_string(0) == b"ok"
    assert b"type" in lib.dp_status_string(-3)
    assert lib.dp_status_string(12345) == b"unknown status"


def test_model_load_without_device_fails_cleanly(model_path):
    """Here there is no GPU: loading must return an error, never fall back to a CPU path."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2602_02234_amd import Model, DPError
    with pytest.raises(DPError):
        Model(model_path)


@pytest.mark.parametrize("prec", [0, 1])
def test_every_weight_pointer_is_bound(model_path, prec):
    """The host-side image check: every weight pointer the kernels of a precision read
    is set and inside the image; clearing any one of them is reported by name."""
    from paper_2602_02234_amd import _lib
    lib = _lib.load()
    nbytes = ctypes.c_size_t(0)
    assert lib.dp_check_model_file(model_path.encode(), prec, None, ctypes.byref(nbytes)) == 0, \
        lib.dp_last_error()
    assert nbytes.value > 4 * 500_000 // (2 if prec else 1)
    names = ["Bt", "F4d", "ebias", "gamma1"] + (["Wqk1", "F1T"] if prec == 0 else ["b16.Wvo0", "b16.F3.lo"])
    for name in names:
        s = lib.dp_check_model_file(model_path.encode(), prec, name.encode(), None)
        assert s == -2, name
        assert name.encode() in lib.dp_last_error()
    assert lib.dp_check_model_file(model_path.encode(), prec, b"no_such_member", None) == -1


def test_truncated_model_file_is_refused(model_path, tmp_path):
    from paper_2602_02234_amd import _lib
    lib = _lib.load()
    raw = open(model_path, "rb").read()
    bad = tmp_path / "short.bin"
    bad.write_bytes(raw[:-8])
    assert lib.dp_check_model_file(str(bad).encode(), 0, None, None) == -2


@pytest.mark.parametrize("prec", [0, 1])
def test_three_head_model_binds_every_head(prec):
    from paper_2602_02234_amd import _lib
    from synth import default_model_file
    lib = _lib.load()
    path = default_model_file(nheads=3).encode()
    assert lib.dp_check_model_file(path, prec, None, None) == 0, lib.dp_last_error()
    for name in (["F1T.2", "ebias.1"] if prec == 0 else ["b16.F3.2.lo", "F4d.2"]):
        assert lib.dp_check_model_file(path, prec, name.encode(), None) == -2, name


def test_gnn_load_without_device_fails_cleanly():
    """The GNN-variant entry point also reports an error without a GPU (no CPU path)."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2602_02234_amd import GnnModel, DPError
    from synth.gnn_weights import default_gnn_file
    with pytest.raises(DPError):
        GnnModel(default_gnn_file())


def test_rep_load_without_device_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2602_02234_amd import RepModel, DPError
    from synth.rep_weights import default_rep_file
    with pytest.raises(DPError):
        RepModel(default_rep_file())
