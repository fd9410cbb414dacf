"""Full-size systems (the 10k-, 25k- and 40k-atom solvated chains) through the device
entry point that bench.py times, checked on sampled atoms against the FP64 oracle.

The oracle evaluates only what the sampled atoms need: their own neighbour lists
(bit-exact), their atomic energies, and the pair gradients of every atom within the
cutoff, which give F_i = sum_j g_ij - sum_j g_ji.  Properties that hold at any size
are checked on the whole system: zero net force and a symmetric virial.
"""
import numpy as np
import pytest

from oracle.dp import evaluate_subset
from oracle.neighbors import neighbor_list_cells
from synth import config_system
from tolerances import TOL

pytestmark = pytest.mark.gpu

SAMPLES = 8


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module", params=["chain10k", "chain25k", "chain40k"])
def system(request):
    return config_system(request.param)


@pytest.fixture(scope="module")
def oracle_lists(omodel, system):
    return neighbor_list_cells(system.coords, system.box, omodel.rc, omodel.sel)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_full_size_sampled_atoms_match_oracle(torch_cuda, gpu_models, omodel, system, oracle_lists, prec):
    torch = torch_cuda
    s = system
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

    nl, nn, _ = oracle_lists
    atoms = np.random.default_rng(5).choice(s.natoms, size=SAMPLES, replace=False)
    gl, gn, _ = gpu.neighbors(s.coords, s.box)
    assert np.array_equal(gn[atoms], nn[atoms])
    assert np.array_equal(gl[atoms], nl[atoms])

    dF, dE, Eref = [], [], []
    for i in atoms:
        centres = [int(i)] + nl[i, :nn[i]].tolist()
        e, nbrs, gs, _ = evaluate_subset(omodel, s.coords, s.types, s.box, centres, nl, nn)
        f = gs[0].sum(0)
        for js, g in zip(nbrs[1:], gs[1:]):
            f = f - g[np.nonzero(js == i)[0][0]]
        dF.append(F[i] - f)
        dE.append(Ei[i] - e[0])
        Eref.append(e[0])
    dF, dE = np.array(dF), np.array(dE)
    tol = TOL[prec]
    m = dict(f_rmse=float(np.sqrt(np.mean(dF ** 2))), f_max=float(np.abs(dF).max()),
             e_atom_rel=float(np.abs(dE).max() / np.abs(Eref).max()))
    print(s.natoms, "atoms", prec, m)
    bad = {k: (v, tol[k]) for k, v in m.items() if not v <= tol[k]}
    assert not bad, f"{prec}: outside tolerance {bad}"

    # any size: the forces sum to zero, the virial is symmetric, E is the sum of the E_i
    scale = np.sqrt(np.mean(F ** 2))
    assert np.abs(F.sum(0)).max() <= tol["f_max"] * scale * np.sqrt(s.natoms)
    assert np.abs(V - V.T).max() <= tol["vir_rel"] * np.abs(V).max()
    assert abs(E.item() - Ei.sum()) <= 1e-9 * abs(E.item())
