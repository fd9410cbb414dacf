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


def _scalar_energies(m, X, types):
    """E_i of an open cluster by plain Python loops over atoms, edges, angles and
    feature components, written from the model's definition (no arrays, no shared code
    with oracle/gnn.py beyond the parameters)."""
    import math
    p = {k: v.tolist() for k, v in m.p.items()}
    N = len(X)

    def dist(i, j):
        return math.sqrt(sum((X[j][a] - X[i][a]) ** 2 for a in range(3)))

    def sw(r, rc):
        if r < m.rcs:
            return 1.0
        if r >= rc:
            return 0.0
        u = (r - m.rcs) / (rc - m.rcs)
        return u ** 3 * (-6 * u * u + 15 * u - 10) + 1

    def lin(x, W, b):
        return [sum(x[q] * W[q][c] for q in range(len(x))) + b[c] for c in range(len(b))]

    nb = {i: [j for j in range(N) if j != i and dist(i, j) < m.rc] for i in range(N)}
    close = {i: [j for j in nb[i] if dist(i, j) < m.rca][:m.asel] for i in range(N)}
    n = {i: list(p["TN"][types[i]]) for i in range(N)}
    e = {(i, j): [math.tanh(sw(dist(i, j), m.rc) / dist(i, j) * p["We0"][0][c] + p["be0"][c]) for c in range(64)]
         for i in range(N) for j in nb[i]}
    a = {}
    for i in range(N):
        for j in close[i]:
            for k in close[i]:
                if j != k:
                    cs = sum((X[j][t] - X[i][t]) * (X[k][t] - X[i][t]) for t in range(3)) / (dist(i, j) * dist(i, k))
                    a[(i, j, k)] = [math.tanh(cs * p["Wa0"][0][c] + p["ba0"][c]) for c in range(32)]
    for l in range(3):
        a1 = {key: [av[c] + math.tanh(z) for c, z in enumerate(
            lin(av + e[key[0], key[1]][:32] + e[key[0], key[2]][:32], p[f"Waa{l}"], p[f"baa{l}"]))]
            for key, av in a.items()}
        msg = {key: [0.0] * 64 for key in e}
        for (i, j, k), av in a1.items():
            wgt = sw(dist(i, j), m.rca) * sw(dist(i, k), m.rca) / m.asel
            z = lin(av + e[i, k][:32], p[f"Wea{l}"], p[f"bea{l}"])
            for c in range(64):
                msg[i, j][c] += wgt * math.tanh(z[c])
        e1 = {(i, j): [ev[c] + math.tanh(z) + msg[i, j][c] for c, z in enumerate(
            lin(n[i] + n[j] + ev, p[f"Wee{l}"], p[f"bee{l}"]))] for (i, j), ev in e.items()}
        n1 = {}
        for i in range(N):
            agg = [sum(sw(dist(i, j), m.rc) * e1[i, j][c] for j in nb[i]) / m.sel for c in range(64)]
            n1[i] = [n[i][c] + math.tanh(z) for c, z in enumerate(lin(n[i] + agg, p[f"Wnn{l}"], p[f"bnn{l}"]))]
        a, e, n = a1, e1, n1
    out = []
    for i in range(N):
        y1 = [math.tanh(z) for z in lin(n[i], p["G1"], p["d1"])]
        y2 = [math.tanh(z) + y1[c] for c, z in enumerate(lin(y1, p["G2"], p["d2"]))]
        out.append(lin(y2, p["G3"], p["d3"])[0])
    return out


def test_scalar_loop_reevaluation(gm):
    """The vectorised forward equals a loop-by-loop evaluation of the model on a 7-atom
    cluster with every pair within rca (42 angles at each atom)."""
    X, t = _cluster(7, 21, spread=1.8, dmin=1.0)
    d = np.sqrt(((X[:, None] - X[None]) ** 2).sum(-1))
    assert d.max() < gm.rca
    ref = np.array(_scalar_energies(gm, X.tolist(), t.tolist()))
    Ei = forward(gm, build_graph(gm, X, t, None))
    assert np.abs(Ei - ref).max() < 1e-9 * np.abs(ref).max()
