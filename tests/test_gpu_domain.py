"""One GPU's share of a spatially decomposed system (dp_compute_owned_device): owned atoms
first, then the ghosts within rc of them.  E_i and g_ij are computed for owned atoms only;
the force rows of ghost atoms are the contributions returned to their owners.

Checks: (1) a 2x2x2 decomposition of a periodic 3k-atom solvated chain, every share on
this GPU, gives back the whole system's E, F and virial (against the FP64 oracle);
(2) the share shape of the 25k-atom system split 8 ways (one of the 8 domains: 3.2k
owned atoms and the 3.8k atoms within rc of them): owned E_i, complete forces of interior owned atoms and the
returned ghost rows, on sampled atoms, against the oracle's pair gradients.
"""
import numpy as np
import pytest
from scipy.spatial import cKDTree

from oracle.dp import evaluate, evaluate_subset
from oracle.neighbors import neighbor_list_cells
from synth import config_system
from tolerances import TOL, compare, assert_within

pytestmark = pytest.mark.gpu


def _domains(s, rc, split=2):
    """Owned atoms of each of split^3 domains (by wrapped position) and their ghosts: the
    other atoms within rc of an owned atom (minimum image)."""
    L = np.diag(s.box)
    w = s.coords % L
    cell = np.minimum((w / (L / split)).astype(int), split - 1)
    dom = (cell[:, 0] * split + cell[:, 1]) * split + cell[:, 2]
    tree = cKDTree(w, boxsize=L)
    out = []
    for d in range(split ** 3):
        owned = np.nonzero(dom == d)[0]
        near = tree.query_ball_point(w[owned], r=rc)
        ghosts = np.setdiff1d(np.unique(np.concatenate([np.asarray(x, dtype=np.int64) for x in near])), owned)
        out.append((owned, ghosts))
    return out


def _run_share(torch, gpu, s, owned, ghosts):
    dev = torch.device("cuda:0")
    idx = np.concatenate([owned, ghosts])
    X = torch.tensor(s.coords[idx], device=dev)
    T = torch.tensor(s.types[idx], device=dev)
    F = torch.zeros((len(idx), 3), dtype=torch.float64, device=dev)
    V = torch.zeros(9, dtype=torch.float64, device=dev)
    E = torch.zeros(1, dtype=torch.float64, device=dev)
    Ei = torch.zeros(len(owned), dtype=torch.float64, device=dev)
    gpu.compute_owned_device(X, T, len(owned), s.box, forces=F, virial=V, energy=E, atom_energy=Ei)
    torch.cuda.synchronize()
    return idx, E.item(), F.cpu().numpy(), V.cpu().numpy().reshape(3, 3), Ei.cpu().numpy()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_eight_shares_recover_the_whole_system(gpu_models, omodel, prec):
    import torch
    s = config_system("chain3k")
    ref = evaluate(omodel, s.coords, s.types, s.box)
    gpu = gpu_models[prec]
    E, F, V, Ei = 0.0, np.zeros_like(s.coords), np.zeros((3, 3)), np.zeros(s.natoms)
    for owned, ghosts in _domains(s, omodel.rc):
        assert len(ghosts) > 0
        idx, e, f, v, ei = _run_share(torch, gpu, s, owned, ghosts)
        E += e
        np.add.at(F, idx, f)
        V += v
        Ei[owned] = ei
    m = compare({"E": E, "F": F, "virial": V, "E_i": Ei}, ref, s.natoms)
    print(prec, m)
    assert_within(m, prec)
    # the whole-system call on the same GPU agrees with the recombined shares
    full = gpu.compute(s.coords, s.types, s.box)
    assert np.max(np.abs(full["F"] - F)) <= TOL[prec]["f_max"]


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_share_of_25k_system(gpu_models, omodel, prec):
    import torch
    s = config_system("chain25k")
    owned, ghosts = _domains(s, omodel.rc)[0]
    print("owned", len(owned), "ghosts", len(ghosts))
    assert 2500 < len(owned) < 3800 and 3000 < len(ghosts) < 6500
    gpu = gpu_models[prec]
    idx, E, F, V, Ei = _run_share(torch, gpu, s, owned, ghosts)
    nl, nn, _ = neighbor_list_cells(s.coords, s.box, omodel.rc, omodel.sel)
    is_owned = np.zeros(s.natoms, dtype=bool)
    is_owned[owned] = True
    rng = np.random.default_rng(9)
    # owned atoms all of whose neighbours are owned: their force is complete in this share
    interior = [i for i in owned if is_owned[nl[i, :nn[i]]].all()]
    pick_i = rng.choice(len(owned), size=16, replace=False)
    pick_int = rng.choice(interior, size=16, replace=False)
    pick_g = rng.choice(len(ghosts), size=16, replace=False)
    tol = TOL[prec]
    # owned E_i
    e, _, _, _ = evaluate_subset(omodel, s.coords, s.types, s.box, owned[pick_i], nl, nn)
    assert np.abs(Ei[pick_i] - e).max() <= tol["e_atom"]
    dF = []
    pos = {int(a): k for k, a in enumerate(idx)}
    for k in list(pick_int) + [int(ghosts[g]) for g in pick_g]:
        # the oracle's share of row k: sum_j g_kj (k owned) - sum_{owned c: k in N(c)} g_ck
        cen = [c for c in [k] + nl[k, :nn[k]].tolist() if is_owned[c]]
        _, nbrs, gs, _ = evaluate_subset(omodel, s.coords, s.types, s.box, cen, nl, nn)
        f = np.zeros(3)
        for c, js, g in zip(cen, nbrs, gs):
            if c == k:
                f += g.sum(0)
            else:
                hit = np.nonzero(js == k)[0]
                if len(hit):
                    f -= g[hit[0]]
        dF.append(F[pos[k]] - f)
    dF = np.array(dF)
    m = dict(f_rmse=float(np.sqrt(np.mean(dF ** 2))), f_max=float(np.abs(dF).max()))
    print(prec, "share of chain25k", m)
    assert m["f_rmse"] <= tol["f_rmse"] and m["f_max"] <= tol["f_max"]
