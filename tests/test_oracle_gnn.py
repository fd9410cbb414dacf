"""Pins of the GNN-variant oracle (oracle/gnn.py), CPU only.

* The hand-written gradient equals central differences of the energy: every atom and
  component of a 40-atom open cluster, and sampled atoms of the 192-atom water box.
* Invariances: rotation of an open cluster, translation with wrap and permutation of the
  periodic water box; forces sum to zero.
* Receptive field of three message-passing layers: on a chain of atoms 4.2 A apart (each
  sees only its two neighbours within rc, none within the angle cutoff), moving atom 0
  changes E_3 and leaves E_4 exactly as it was.
* Angles: on a cluster where some neighbours are within rca = 4 A, switching the angle
  terms off (their message weights at zero) changes the energy, and a neighbour moved
  radially through rca changes it smoothly.
* Smoothness through rc.
"""
import numpy as np
import pytest

from oracle.gnn import load_gnn_model, evaluate, energy, forward, build_graph
from synth.gnn_weights import default_gnn_file


@pytest.fixture(scope="module")
def gm():
    return load_gnn_model(default_gnn_file())


def _cluster(n, seed, spread, dmin=1.0):
    rng = np.random.default_rng(seed)
    X = []
    while len(X) < n:
        p = rng.uniform(-spread, spread, size=3)
        if all(np.linalg.norm(p - q) > dmin for q in X):
            X.append(p)
    return np.array(X), rng.integers(0, 5, size=n).astype(np.int32)


def test_force_scale_gives_unit_rms(gm, water192):
    r = evaluate(gm, water192.coords, water192.types, water192.box)
    assert abs(np.sqrt(np.mean(r["F"] ** 2)) - 1.0) < 1e-6
    assert np.abs(r["F"].sum(0)).max() < 1e-10
    v = r["virial"]
    assert np.abs(v - v.T).max() < 1e-9 * np.abs(v).max()


def test_gradient_equals_central_differences_cluster(gm):
    X, t = _cluster(40, 3, spread=5.0)
    r = evaluate(gm, X, t, None)
    h = 1e-5
    fd = np.zeros_like(X)
    for i in range(len(X)):
        for a in range(3):
            Xp = X.copy(); Xp[i, a] += h
            Xm = X.copy(); Xm[i, a] -= h
            fd[i, a] = -(energy(gm, Xp, t, None) - energy(gm, Xm, t, None)) / (2 * h)
    err = np.abs(fd - r["F"]).max()
    print("cluster max |FD - F|", err, "max |F|", np.abs(r["F"]).max())
    assert err < 2e-6 * max(1.0, np.abs(r["F"]).max())


def test_gradient_equals_central_differences_water(gm, water192):
    s = water192
    r = evaluate(gm, s.coords, s.types, s.box)
    h = 1e-5
    rng = np.random.default_rng(4)
    for i in rng.choice(s.natoms, size=3, replace=False):
        a = int(rng.integers(3))
        Xp = s.coords.copy(); Xp[i, a] += h
        Xm = s.coords.copy(); Xm[i, a] -= h
        fd = -(energy(gm, Xp, s.types, s.box) - energy(gm, Xm, s.types, s.box)) / (2 * h)
        assert abs(fd - r["F"][i, a]) < 2e-5, (i, a, fd, r["F"][i, a])


def test_rotation_invariance(gm):
    X, t = _cluster(30, 5, spread=4.5)
    q = np.random.default_rng(8).normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    R = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                  [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                  [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])
    a = evaluate(gm, X, t, None)
    b = evaluate(gm, X @ R.T, t, None)
    assert abs(a["E"] - b["E"]) < 1e-9 * abs(a["E"])
    assert np.abs(a["F"] @ R.T - b["F"]).max() < 1e-9


def test_translation_and_permutation(gm, water192):
    s = water192
    a = evaluate(gm, s.coords, s.types, s.box)
    b = evaluate(gm, s.coords + np.array([3.3, -7.1, 20.0]), s.types, s.box)
    assert abs(a["E"] - b["E"]) < 1e-9 * abs(a["E"])
    perm = np.random.default_rng(2).permutation(s.natoms)
    c = evaluate(gm, s.coords[perm], s.types[perm], s.box)
    assert abs(a["E"] - c["E"]) < 1e-9 * abs(a["E"])
    assert np.abs(a["F"][perm] - c["F"]).max() < 1e-9


def test_receptive_field_is_three_hops(gm):
    X = np.array([[4.2 * k, 0.0, 0.0] for k in range(7)])
    t = np.array([0, 1, 2, 3, 4, 0, 1], dtype=np.int32)
    g0 = build_graph(gm, X, t, None)
    assert len(g0["ep"]) == 0  # no neighbours within the angle cutoff
    E0 = forward(gm, g0)
    X1 = X.copy()
    X1[0] += np.array([0.3, 0.2, -0.1])
    E1 = forward(gm, build_graph(gm, X1, t, None))
    assert abs(E1[3] - E0[3]) > 1000 * np.spacing(abs(E0[3]))  # well above rounding
    assert np.array_equal(E1[4:], E0[4:])


def test_angles_enter_and_are_smooth(gm):
    X, t = _cluster(12, 9, spread=2.5, dmin=1.2)
    g = build_graph(gm, X, t, None)
    assert len(g["ep"]) > 50
    E = forward(gm, g).sum()
    g2 = dict(g)
    g2["ep"] = g["ep"][:0]
    g2["eq"] = g["eq"][:0]
    assert abs(forward(gm, g2).sum() - E) > 1e-3
    # move one neighbour of atom 0 radially through rca: energy continuous, no jump
    d = X[1] - X[0]
    u = d / np.linalg.norm(d)
    rs = np.arange(3.95, 4.05, 0.001)
    Es = []
    for rr in rs:
        Y = X.copy()
        Y[1] = X[0] + u * rr
        Es.append(energy(gm, Y, t, None))
    jumps = np.abs(np.diff(np.diff(Es)))
    assert jumps.max() < 1e-5


def test_smooth_through_cutoff(gm):
    X = np.array([[0.0, 0.0, 0.0], [1.0, 0.5, 0.0], [-0.8, 0.9, 0.3], [5.9, 0.0, 0.0]])
    t = np.array([0, 1, 2, 3], dtype=np.int32)
    Es = []
    for rr in np.arange(5.98, 6.02, 0.001):
        Y = X.copy()
        Y[3, 0] = rr
        Es.append(energy(gm, Y, t, None))
    assert np.abs(np.diff(np.diff(Es))).max() < 1e-6


def test_last_layer_norm(gm):
    """||G3||_2 of the seeded GNN model, the constant the energy bounds of the GPU paths use."""
    from tolerances import G3NORM
    assert abs(np.linalg.norm(gm.p["G3"]) - G3NORM) < 0.05
