"""Central finite differences of the oracle's energy against its hand-written gradient
on every atom of the 192-atom water box and on 32 seeded atoms of each solvated chain
(10k, 25k and 40k atoms), h = 1e-4 A, plus a Richardson pair (CPU only).

For a chain atom i only the energies of i and its neighbours change when i moves,
and those depend only on atoms within 2 rc of i.  The finite differences therefore
run on that cluster, cut out of the periodic box around i (minimum image, open
boundaries), and compare with F_i from the oracle's pair gradients on the same
cluster.  The water box (12.4 A) is smaller than such a cluster, so there the
energy of i's neighbourhood is evaluated in the periodic box itself.
"""
import concurrent.futures as cf
import multiprocessing as mp

import numpy as np
import pytest

from oracle.dp import evaluate_subset, local_energy
from oracle.neighbors import neighbor_list_cells

H = 1e-4


def _cluster_fd(args):
    """(F_i,a from the gradient, FD at h, Richardson from h and 2h) for one chain atom."""
    from threadpoolctl import threadpool_limits
    m, X, types, L, i, a = args
    with threadpool_limits(limits=1):
        d = X - X[i]
        d -= L * np.rint(d / L)
        keep = np.nonzero(np.sum(d * d, axis=1) < (2 * m.rc + 0.5) ** 2)[0]
        Xc, tc = d[keep], types[keep]
        ic = int(np.nonzero(keep == i)[0][0])
        nl, nn, _ = neighbor_list_cells(Xc, None, m.rc, m.sel)
        centres = [ic] + nl[ic, :nn[ic]].tolist()
        _, nbrs, gs, _ = evaluate_subset(m, Xc, tc, None, centres, nl, nn)
        f = gs[0].sum(0)
        for js, g in zip(nbrs[1:], gs[1:]):
            f = f - g[np.nonzero(js == ic)[0][0]]

        def fd(h):
            Xp = Xc.copy(); Xp[ic, a] += h
            Xm = Xc.copy(); Xm[ic, a] -= h
            return -(local_energy(m, Xp, tc, None, centres) - local_energy(m, Xm, tc, None, centres)) / (2 * h)

        f1, f2 = fd(H), fd(2 * H)
    return float(f[a]), f1, (4 * f1 - f2) / 3


def _water_fd(args):
    from threadpoolctl import threadpool_limits
    m, X, types, box, atoms, i, a = args
    with threadpool_limits(limits=1):
        Xp = X.copy(); Xp[i, a] += H
        Xm = X.copy(); Xm[i, a] -= H
        return -(local_energy(m, Xp, types, box, atoms) - local_energy(m, Xm, types, box, atoms)) / (2 * H)


def _pool():
    return cf.ProcessPoolExecutor(max_workers=min(8, mp.cpu_count()), mp_context=mp.get_context("fork"))


def test_fd_every_atom_water192(omodel, water192, oracle_water192):
    s = water192
    nl, nn, _ = neighbor_list_cells(s.coords, s.box, omodel.rc + 0.01, 400)
    jobs = [(omodel, s.coords, s.types, s.box, [i] + nl[i, :nn[i]].tolist(), i, a)
            for i in range(s.natoms) for a in range(3)]
    with _pool() as ex:
        fd = np.array(list(ex.map(_water_fd, jobs, chunksize=8))).reshape(s.natoms, 3)
    err = np.abs(fd - oracle_water192["F"])
    print("water192 all atoms: max |FD - F|", err.max(), "RMS", np.sqrt(np.mean(err ** 2)))
    # O(h^2) truncation (~1e-8 here) plus the float64 noise of a sum of ~90 atomic
    # energies of O(700) eV over 2h (~1e-7): measured max 1.6e-7
    assert err.max() < 5e-7


@pytest.mark.parametrize("name", ["chain10k", "chain25k", "chain40k"])
def test_fd_32_atoms_solvated_chain(omodel, name):
    from synth import config_system
    s = config_system(name)
    L = np.diag(s.box)
    rng = np.random.default_rng(5)
    atoms = rng.choice(s.natoms, size=32, replace=False)
    comps = rng.integers(0, 3, size=32)
    jobs = [(omodel, s.coords, s.types, L, int(i), int(a)) for i, a in zip(atoms, comps)]
    with _pool() as ex:
        res = np.array(list(ex.map(_cluster_fd, jobs)))
    f, fd, rich = res[:, 0], res[:, 1], res[:, 2]
    print(name, "max |FD - F|", np.abs(fd - f).max(), "Richardson", np.abs(rich - f).max(),
          "max |F|", np.abs(f).max())
    # as for the water box (measured 0.9-1.3e-7); Richardson removes the h^2 term but
    # not the noise, which dominates at h = 1e-4
    assert np.abs(fd - f).max() < 5e-7
    assert np.abs(rich - f).max() < 5e-7
