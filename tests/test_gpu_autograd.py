"""The torch.autograd.Function over the library's hand-written backward, and finite differences.

Finite differences of the GPU's own float32-path energy are limited by the
rounding noise of the per-atom energies (about 1e-6 of |E_i| ~ 700 eV, i.e.
~7e-4 eV, summed over the ~90 atoms a displacement touches): at h = 1e-4 A
that noise is ~7e-3 eV / 2e-4 A ~ 30 eV/A, so a plain h = 1e-4 difference of
the float32 energy says nothing; h = 1e-4 is checked on the float64 oracle
instead (tests/test_oracle_physics.py).  Here a Richardson pair at
h = 2e-2 / 1e-2 cancels the O(h^2) truncation; its noise is ~7e-3/1e-2 ~ 0.5
eV/A, so the bound is 1 eV/A -- a check that the library's forces are the
gradient of the library's energy (sign, factor, missing term), not an
accuracy test.  The accuracy test is against the oracle's forces.
"""
import numpy as np
import pytest

from oracle.dp import evaluate
from oracle.neighbors import neighbor_list_cells
from synth import config_system
from tolerances import FP32

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


def test_autograd_forces_equal_library_forces(torch_cuda, gpu_fp32, water192, oracle_water192):
    torch = torch_cuda
    from paper_2602_02234_amd import energy
    s = water192
    x = torch.tensor(s.coords, dtype=torch.float64, device="cuda", requires_grad=True)
    t = torch.tensor(s.types, dtype=torch.int32, device="cuda")
    E = energy(gpu_fp32, x, t, s.box)
    E.backward()
    F_auto = -x.grad.cpu().numpy()
    F_lib = gpu_fp32.compute(s.coords, s.types, s.box)["F"]
    assert np.max(np.abs(F_auto - F_lib)) <= 1e-12 * max(1.0, np.max(np.abs(F_lib)))
    rmse = np.sqrt(np.mean((F_auto - oracle_water192["F"]) ** 2))
    assert rmse <= 1e-5
    assert abs(float(E.item()) - oracle_water192["E"]) <= FP32["e_per_atom"] * s.natoms


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_interleaved_energies_backward_their_own_forward(torch_cuda, gpu_models, prec):
    """Two energy() graphs on one model, differentiated in the opposite order: each
    backward gives the gradient at its own coordinates."""
    torch = torch_cuda
    from paper_2602_02234_amd import energy
    gpu = gpu_models[prec]
    s = config_system("water192")
    t = torch.tensor(s.types, dtype=torch.int32, device="cuda")
    x1 = torch.tensor(s.coords, dtype=torch.float64, device="cuda", requires_grad=True)
    x2 = torch.tensor(s.coords + 0.05, dtype=torch.float64, device="cuda", requires_grad=True)
    x2.data[3, 1] += 0.2
    E1 = energy(gpu, x1, t, s.box)
    E2 = energy(gpu, x2, t, s.box)
    E1.backward()
    E2.backward()
    F1 = gpu.compute(s.coords, s.types, s.box)["F"]
    F2 = gpu.compute(x2.detach().cpu().numpy(), s.types, s.box)["F"]
    for g, F in ((x1.grad, F1), (x2.grad, F2)):
        assert np.max(np.abs(-g.cpu().numpy() - F)) <= 1e-12 * max(1.0, np.max(np.abs(F)))
    assert np.max(np.abs(F1 - F2)) > 1e-3


def test_autograd_upstream_gradient_scales(torch_cuda, gpu_bf16, water192):
    torch = torch_cuda
    from paper_2602_02234_amd import energy
    s = water192
    t = torch.tensor(s.types, dtype=torch.int32, device="cuda")
    x1 = torch.tensor(s.coords, dtype=torch.float64, device="cuda", requires_grad=True)
    energy(gpu_bf16, x1, t, s.box).backward()
    x2 = torch.tensor(s.coords, dtype=torch.float64, device="cuda", requires_grad=True)
    (-2.5 * energy(gpu_bf16, x2, t, s.box)).backward()
    assert torch.allclose(x2.grad, -2.5 * x1.grad, rtol=1e-12, atol=1e-12)


def _local_energy(model, X, types, box, atoms):
    out = model.compute(X, types, box, forces=False, atom_energy=True)
    return float(np.sum(out["E_i"][atoms]))


def test_central_differences_of_gpu_energy(gpu_fp32, omodel):
    s = config_system("chain1k")
    out = gpu_fp32.compute(s.coords, s.types, s.box)
    nl, nn, _ = neighbor_list_cells(s.coords, s.box, 6.2, 400)
    rng = np.random.default_rng(7)
    worst_rich, scale = 0.0, 0.0
    for i in rng.choice(s.natoms, size=32, replace=False):
        atoms = np.array([i] + nl[i, :nn[i]].tolist())
        a = int(rng.integers(3))

        def fd(h):
            Xp = s.coords.copy(); Xp[i, a] += h
            Xm = s.coords.copy(); Xm[i, a] -= h
            return -(_local_energy(gpu_fp32, Xp, s.types, s.box, atoms)
                     - _local_energy(gpu_fp32, Xm, s.types, s.box, atoms)) / (2 * h)

        f = out["F"][i, a]
        worst_rich = max(worst_rich, abs((4 * fd(1e-2) - fd(2e-2)) / 3 - f))
        scale = max(scale, abs(f))
    print("fd richardson worst:", worst_rich, "max |F| sampled:", scale)
    assert worst_rich < 1.0


def test_backward_without_forward_is_an_error(torch_cuda, gpu_fp32):
    torch = torch_cuda
    from paper_2602_02234_amd import DPError
    g = torch.zeros((4, 3), dtype=torch.float64, device="cuda")
    gE = torch.ones(1, dtype=torch.float64, device="cuda")
    gpu_fp32.compute(np.zeros((2, 3)) + np.array([[0, 0, 0], [1.5, 0, 0]]), np.array([0, 1]), None)
    with pytest.raises(DPError, match="DP_ERR_ARG"):
        gpu_fp32.backward_device(gE, g)
