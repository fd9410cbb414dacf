"""dp_compute_device_noalloc (workspace in a static device array, no allocation) against
dp_compute_device on the same inputs: two calls in a row, the second on a smaller
system, in both precisions, called through the C ABI.  The two entry points run the
same kernels, so their results must agree bit for bit; a system above the array's
capacity is refused."""
import ctypes as C

import numpy as np
import pytest

from synth import config_system

pytestmark = pytest.mark.gpu


def _run(lib, model, fn, s, torch, dev):
    X = torch.tensor(s.coords, device=dev)
    T = torch.tensor(s.types, device=dev)
    F = torch.full((s.natoms, 3), np.nan, dtype=torch.float64, device=dev)
    V = torch.full((9,), np.nan, dtype=torch.float64, device=dev)
    E = torch.full((1,), np.nan, dtype=torch.float64, device=dev)
    Ei = torch.full((s.natoms,), np.nan, dtype=torch.float64, device=dev)
    box = np.ascontiguousarray(s.box, dtype=np.float64)
    st = torch.cuda.current_stream(dev).cuda_stream
    p = lambda t: C.c_void_p(t.data_ptr())
    rc = getattr(lib, fn)(model._h, s.natoms, p(X), p(T), C.c_void_p(box.ctypes.data), p(E), p(F), p(V), p(Ei),
                          C.c_void_p(st))
    torch.cuda.synchronize()
    return rc, E.item(), F.cpu().numpy(), V.cpu().numpy(), Ei.cpu().numpy()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_noalloc_equals_allocating_entry_point(model_path, prec):
    import torch
    from paper_2602_02234_amd import Model, _lib
    lib = _lib.load()
    dev = torch.device("cuda:0")
    m = Model(model_path, prec)
    for name in ("chain1k", "water192"):   # the second call is the smaller system
        s = config_system(name)
        ref = _run(lib, m, "dp_compute_device", s, torch, dev)
        got = _run(lib, m, "dp_compute_device_noalloc", s, torch, dev)
        assert ref[0] == 0 and got[0] == 0, (name, got[0], lib.dp_last_error())
        assert got[1] == ref[1], name
        for a, b in zip(got[2:], ref[2:]):
            assert np.array_equal(a, b), name
    big = config_system("chain3k")
    rc = _run(lib, m, "dp_compute_device_noalloc", big, torch, dev)[0]
    assert rc == -8 and b"DP_NOALLOC_MAX_ATOMS" in lib.dp_last_error()
    m.close()
