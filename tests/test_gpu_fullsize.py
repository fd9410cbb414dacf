"""Full-size systems (the 10k-, 25k- and 40k-atom solvated chains) through the device
entry point that bench.py times, checked on sampled atoms against the FP64 oracle.

The oracle evaluates only what the sampled atoms need: their own neighbour lists
(bit-exact), their atomic energies, and the pair gradients of every atom within the
cutoff, which give F_i = sum_j g_ij - sum_j g_ji.  The 32 sampled atoms (seed 5) are
the ones whose oracle forces tests/test_oracle_fd_configs.py checks by central
differences at h = 1e-4 A, so the GPU forces are compared with a gradient that is
itself pinned to finite differences.  The 40k system also goes through the
torch.autograd.Function (hand-written backward).  Properties that hold at any size
are checked on the whole system: zero net force, a symmetric virial, E = sum E_i.
"""
import numpy as np
import pytest

from oracle.dp import evaluate_subset
from oracle.neighbors import neighbor_list_cells
from synth import config_system
from tolerances import TOL

pytestmark = pytest.mark.gpu

SAMPLES = 32


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module", params=["chain10k", "chain25k", "chain40k"])
def system(request):
    return request.param, config_system(request.param)


@pytest.fixture(scope="module")
def oracle_ref(omodel, system):
    """Lists of the whole system, and E_i, F_i of the sampled atoms, from the oracle."""
    _, s = system
    nl, nn, _ = neighbor_list_cells(s.coords, s.box, omodel.rc, omodel.sel)
    atoms = np.random.default_rng(5).choice(s.natoms, size=SAMPLES, replace=False)
    F, E = [], []
    for i in atoms:
        centres = [int(i)] + nl[i, :nn[i]].tolist()
        e, nbrs, gs, _ = evaluate_subset(omodel, s.coords, s.types, s.box, centres, nl, nn)
        f = gs[0].sum(0)
        for js, g in zip(nbrs[1:], gs[1:]):
            f = f - g[np.nonzero(js == i)[0][0]]
        F.append(f)
        E.append(e[0])
    return dict(nl=nl, nn=nn, atoms=atoms, F=np.array(F), E=np.array(E))


def _metrics(F, Ei, ref):
    dF = F[ref["atoms"]] - ref["F"]
    m = dict(f_rmse=float(np.sqrt(np.mean(dF ** 2))), f_max=float(np.abs(dF).max()))
    if Ei is not None:
        m["e_atom"] = float(np.abs(Ei[ref["atoms"]] - ref["E"]).max())
    return m


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_full_size_sampled_atoms_match_oracle(torch_cuda, gpu_models, system, oracle_ref, prec):
    torch = torch_cuda
    name, s = system
    gpu = gpu_models[prec]
    dev = torch.device("cuda:0")
    X = torch.tensor(s.coords, device=dev)
    T = torch.tensor(s.types, device=dev)
    F = torch.zeros((s.natoms, 3), dtype=torch.float64, device=dev)
    V = torch.zeros(9, dtype=torch.float64, device=dev)
    E = torch.zeros(1, dtype=torch.float64, device=dev)
    Ei = torch.zeros(s.natoms, dtype=torch.float64, device=dev)
    gpu.compute_device(X, T, s.box, forces=F, virial=V, energy=E, atom_energy=Ei)
    torch.cuda.synchronize()
    F, V, Ei = F.cpu().numpy(), V.cpu().numpy().reshape(3, 3), Ei.cpu().numpy()
    assert np.isfinite(F).all() and np.isfinite(V).all() and np.isfinite(Ei).all()

    atoms = oracle_ref["atoms"]
    gl, gn, _ = gpu.neighbors(s.coords, s.box)
    assert np.array_equal(gn, oracle_ref["nn"])
    assert np.array_equal(gl, oracle_ref["nl"])

    tol = TOL[prec]
    m = _metrics(F, Ei, oracle_ref)
    print(name, s.natoms, "atoms", prec, m)
    bad = {k: (v, tol[k]) for k, v in m.items() if not v <= tol[k]}
    assert not bad, f"{prec}: outside tolerance {bad}"

    # any size: the forces sum to zero, the virial is symmetric, E is the sum of the E_i
    scale = np.sqrt(np.mean(F ** 2))
    assert np.abs(F.sum(0)).max() <= tol["f_max"] * scale * np.sqrt(s.natoms)
    assert np.abs(V - V.T).max() <= tol["vir_rel"] * np.abs(V).max()
    assert abs(E.item() - Ei.sum()) <= 1e-9 * abs(E.item())

    if name == "chain40k":
        # -dE/dx through DPEnergy: the energy pass, then the library's backward
        from paper_2602_02234_amd import energy
        x = torch.tensor(s.coords, dtype=torch.float64, device=dev, requires_grad=True)
        energy(gpu, x, T, s.box).backward()
        Fa = -x.grad.cpu().numpy()
        m = _metrics(Fa, None, oracle_ref)
        print(name, "autograd", prec, m)
        bad = {k: (v, tol[k]) for k, v in m.items() if not v <= tol[k]}
        assert not bad, f"{prec} autograd: outside tolerance {bad}"
