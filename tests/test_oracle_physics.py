"""Pins of the oracle's gradient, virial, invariances, smoothness and dynamics (CPU only)."""
import numpy as np
import pytest

from oracle.dp import evaluate, energy_only, local_energy
from oracle.neighbors import neighbor_list_cells
from oracle.nve import maxwell_boltzmann, run_nve


def _fd_force(m, s, i, a, h):
    """-dE/dx_ia by central differences over the atoms whose energy can change (i and its neighbours)."""
    nl, nn, _ = neighbor_list_cells(s.coords, s.box, m.rc + 0.01, 400)
    atoms = [i] + nl[i, :nn[i]].tolist()
    Xp = s.coords.copy(); Xp[i, a] += h
    Xm = s.coords.copy(); Xm[i, a] -= h
    return -(local_energy(m, Xp, s.types, s.box, atoms) - local_energy(m, Xm, s.types, s.box, atoms)) / (2 * h)


def test_forces_match_central_differences(omodel, water192, oracle_water192):
    s = water192
    rng = np.random.default_rng(3)
    worst_fd, worst_rich = 0.0, 0.0
    for i in rng.choice(s.natoms, size=6, replace=False):
        for a in range(3):
            f0 = _fd_force(omodel, s, int(i), a, 1e-4)
            f1 = _fd_force(omodel, s, int(i), a, 1e-3)
            f2 = _fd_force(omodel, s, int(i), a, 5e-4)
            rich = (4 * f2 - f1) / 3
            worst_fd = max(worst_fd, abs(f0 - oracle_water192["F"][i, a]))
            worst_rich = max(worst_rich, abs(rich - oracle_water192["F"][i, a]))
    print(worst_fd, worst_rich)
    # h = 1e-4: O(h^2) truncation plus float64 noise of O(1e3) eV atomic energies over 2h
    assert worst_fd < 2e-6
    # Richardson on (1e-3, 5e-4) cancels the h^2 term; the h^4 term and the noise stay below 1e-7
    assert worst_rich < 1e-7


def test_net_force_zero_and_virial_symmetric(oracle_water192):
    assert np.max(np.abs(oracle_water192["F"].sum(0))) < 1e-10
    v = oracle_water192["virial"]
    assert np.max(np.abs(v - v.T)) < 1e-10 * np.max(np.abs(v))


def test_virial_diagonal_by_box_strain(omodel, water192, oracle_water192):
    """dE/d eps_aa = -Xi_aa when coordinates and box edge a are scaled by (1 + eps)."""
    s = water192
    h = 1e-4        # total energies are O(1e5) eV: smaller steps drown in float64 rounding
    for a in range(3):
        sc = np.ones(3); sc[a] += h
        Ep = energy_only(omodel, s.coords * sc, s.types, s.box * sc)
        sc = np.ones(3); sc[a] -= h
        Em = energy_only(omodel, s.coords * sc, s.types, s.box * sc)
        dE = (Ep - Em) / (2 * h)
        assert abs(dE + oracle_water192["virial"][a, a]) < 1e-5 * max(1.0, abs(dE))


def _cluster(n=40, seed=0):
    rng = np.random.default_rng(seed)
    X = []
    while len(X) < n:
        p = rng.uniform(-6, 6, size=3)
        if all(np.linalg.norm(p - q) > 1.0 for q in X):
            X.append(p)
    return np.array(X), rng.integers(0, 5, size=n).astype(np.int32)


def test_virial_off_diagonal_open_cluster(omodel):
    X, t = _cluster(24, 1)
    out = evaluate(omodel, X, t, None)
    h = 1e-4
    for a, b in ((0, 1), (1, 2), (2, 0)):
        eps = np.zeros((3, 3)); eps[a, b] = h
        Ep = energy_only(omodel, X @ (np.eye(3) + eps).T, t, None)
        Em = energy_only(omodel, X @ (np.eye(3) - eps).T, t, None)
        dE = (Ep - Em) / (2 * h)            # dE/d eps_ab = sum g_a Delta_b = -Xi_ba
        assert abs(dE + out["virial"][b, a]) < 1e-6 * max(1.0, abs(dE))


def test_translation_and_wrap_invariance(omodel, water192, oracle_water192):
    s = water192
    L = s.box[0, 0]
    X2 = (s.coords + np.array([3.3, -7.1, 11.9])) % L
    o2 = evaluate(omodel, X2, s.types, s.box)
    assert abs(o2["E"] - oracle_water192["E"]) < 1e-10 * abs(o2["E"])
    assert np.max(np.abs(o2["F"] - oracle_water192["F"])) < 1e-9


def test_permutation_invariance(omodel, water192, oracle_water192):
    s = water192
    perm = np.random.default_rng(2).permutation(s.natoms)
    o2 = evaluate(omodel, s.coords[perm], s.types[perm], s.box)
    assert abs(o2["E"] - oracle_water192["E"]) < 1e-10 * abs(o2["E"])
    assert np.max(np.abs(o2["F"] - oracle_water192["F"][perm])) < 1e-9


def test_rotation_invariance_open_cluster(omodel):
    X, t = _cluster(40, 4)
    o1 = evaluate(omodel, X, t, None)
    q = np.random.default_rng(5).normal(size=4); q /= np.linalg.norm(q)
    w, x, y, z = q
    R = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                  [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                  [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])
    o2 = evaluate(omodel, X @ R.T, t, None)
    assert abs(o2["E"] - o1["E"]) < 1e-10 * abs(o1["E"])
    assert np.max(np.abs(o2["F"] - o1["F"] @ R.T)) < 1e-9
    assert np.max(np.abs(o2["virial"] - R @ o1["virial"] @ R.T)) < 1e-9


def test_cubic_box_axis_permutation(omodel, water192, oracle_water192):
    s = water192
    P = [2, 0, 1]
    o2 = evaluate(omodel, s.coords[:, P], s.types, s.box)
    assert abs(o2["E"] - oracle_water192["E"]) < 1e-10 * abs(o2["E"])
    assert np.max(np.abs(o2["F"] - oracle_water192["F"][:, P])) < 1e-9


def test_smooth_through_cutoff(omodel):
    """Move one atom radially through rc: energy has no jump beyond its local slope."""
    X, t = _cluster(12, 6)
    d = np.array([1.0, 0.3, -0.2]); d /= np.linalg.norm(d)
    rs = np.arange(5.95, 6.05, 1e-3)
    Es = []
    for r in rs:
        Y = np.vstack([X, [X[0] + r * d]])
        Es.append(energy_only(omodel, Y, np.append(t, 1), None))
    Es = np.array(Es)
    # A jump J in E (or in dE/dr times the step) at rc would put a second difference of size ~J
    # there; for a C2 energy the second differences are h^2 E'' and vary smoothly through rc.
    d2 = np.abs(np.diff(Es, 2))
    assert np.max(d2) < 3.0 * np.median(d2[d2 > 0]) + 1e-12


def test_pair_energy_flattens_at_cutoff(omodel):
    """Two atoms: E(r) reaches its separated value at rc with zero slope (C2 switch)."""
    t = np.array([0, 2], dtype=np.int32)

    def E(r):
        return energy_only(omodel, np.array([[0.0, 0.0, 0.0], [r, 0.0, 0.0]]), t, None)

    E_far = E(6.5)
    assert E(6.0) == E_far
    # the pair term enters through the descriptor quadratically in s ~ (rc - r)^3 near rc
    assert abs(E(6.0 - 1e-2) - E_far) < 1e-12
    assert abs(E(4.0) - E_far) > 1e-6


@pytest.mark.slow
def test_nve_drift_second_order(omodel):
    """Velocity Verlet: halving dt cuts the energy error about fourfold."""
    X, t = _cluster(18, 9)
    v = maxwell_boltzmann(t, 300.0, seed=1)
    e1 = run_nve(omodel, X, t, None, v, dt=0.5, steps=16)
    e2 = run_nve(omodel, X, t, None, v, dt=0.25, steps=32)
    err1 = np.max(np.abs(e1 - e1[0]))
    err2 = np.max(np.abs(e2 - e2[0]))
    assert err1 < 5e-3 * len(t)
    assert 2.5 < err1 / err2 < 6.0
