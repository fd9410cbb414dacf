"""Pins of the repformer-style oracle (oracle/repformer.py), CPU only.

* The hand-written gradient equals central differences of the energy: every coordinate
  of a 30-atom open cluster, and sampled atoms of the 192-atom water box.
* A loop-by-loop evaluation of the model (written from its definition) equals the
  vectorised forward on a small cluster.
* Invariances: rotation of an open cluster, translation with wrap and permutation of
  the water box; forces sum to zero; the virial is symmetric.
* Receptive field of three layers: on a chain of atoms 4.2 A apart, moving atom 0
  changes E_3 and leaves E_4 exactly as it was.
* Smoothness as a neighbour crosses rc (attention weights, convolution and contraction
  all carry the switch).
"""
import math

import numpy as np
import pytest

from oracle.repformer import build_edges, energy, evaluate, forward, load_rep_model
from synth.rep_weights import default_rep_file


@pytest.fixture(scope="module")
def rm():
    return load_rep_model(default_rep_file())


def _cluster(n, seed, spread, dmin=1.0):
    rng = np.random.default_rng(seed)
    X = []
    while len(X) < n:
        p = rng.uniform(-spread, spread, size=3)
        if all(np.linalg.norm(p - q) > dmin for q in X):
            X.append(p)
    return np.array(X), rng.integers(0, 5, size=n).astype(np.int32)


def test_force_scale_and_invariants_water(rm, water192):
    r = evaluate(rm, water192.coords, water192.types, water192.box)
    assert abs(np.sqrt(np.mean(r["F"] ** 2)) - 1.0) < 1e-6
    assert np.abs(r["F"].sum(0)).max() < 1e-9
    v = r["virial"]
    assert np.abs(v - v.T).max() < 1e-9 * np.abs(v).max()


def test_gradient_equals_central_differences_cluster(rm):
    X, t = _cluster(30, 3, spread=4.5)
    r = evaluate(rm, X, t, None)
    h = 1e-5
    fd = np.zeros_like(X)
    for i in range(len(X)):
        for a in range(3):
            Xp = X.copy(); Xp[i, a] += h
            Xm = X.copy(); Xm[i, a] -= h
            fd[i, a] = -(energy(rm, Xp, t, None) - energy(rm, Xm, t, None)) / (2 * h)
    err = np.abs(fd - r["F"]).max()
    print("cluster max |FD - F|", err, "max |F|", np.abs(r["F"]).max())
    assert err < 2e-5 * max(1.0, np.abs(r["F"]).max())


def test_gradient_equals_central_differences_water(rm, water192):
    s = water192
    r = evaluate(rm, s.coords, s.types, s.box)
    h = 1e-5
    rng = np.random.default_rng(4)
    for i in rng.choice(s.natoms, size=4, replace=False):
        a = int(rng.integers(3))
        Xp = s.coords.copy(); Xp[i, a] += h
        Xm = s.coords.copy(); Xm[i, a] -= h
        fd = -(energy(rm, Xp, s.types, s.box) - energy(rm, Xm, s.types, s.box)) / (2 * h)
        assert abs(fd - r["F"][i, a]) < 2e-4, (i, a, fd, r["F"][i, a])


def _scalar_energies(m, X, types):
    """E_i by plain Python loops, written from the model's definition."""
    p = {k: v.tolist() for k, v in m.p.items()}
    N = len(X)

    def vec(i, j):
        return [X[j][a] - X[i][a] for a in range(3)]

    def norm(v):
        return math.sqrt(sum(x * x for x in v))

    def sw(r):
        if r < m.rcs:
            return 1.0
        if r >= m.rc:
            return 0.0
        u = (r - m.rcs) / (m.rc - m.rcs)
        return u ** 3 * (-6 * u * u + 15 * u - 10) + 1

    def lin(x, W, b=None):
        return [sum(x[q] * W[q][c] for q in range(len(x))) + (b[c] if b else 0.0) for c in range(len(W[0]))]

    nb = {i: [j for j in range(N) if j != i and norm(vec(i, j)) < m.rc] for i in range(N)}
    g1 = {i: list(p["TN"][types[i]]) for i in range(N)}
    g2 = {}
    for i in range(N):
        for j in nb[i]:
            r = norm(vec(i, j))
            g2[i, j] = [math.tanh(sw(r) / r * p["Wp0"][0][c] + p["bp0"][c]) for c in range(32)]
    for l in range(3):
        g2a = {(i, j): [v[c] + math.tanh(z) for c, z in enumerate(lin(v + g1[j], p[f"Wa{l}"], p[f"ba{l}"]))]
               for (i, j), v in g2.items()}
        g2b = {}
        for i in range(N):
            Q = {j: lin(g2a[i, j], p[f"Wq{l}"]) for j in nb[i]}
            K = {j: lin(g2a[i, j], p[f"Wk{l}"]) for j in nb[i]}
            V = {j: lin(g2a[i, j], p[f"Wv{l}"]) for j in nb[i]}
            for j in nb[i]:
                w = {k: sw(norm(vec(i, k))) * math.exp(sum(Q[j][c] * K[k][c] for c in range(32)) / math.sqrt(32))
                     for k in nb[i]}
                Z = sum(w.values())
                hj = [x / norm(vec(i, j)) for x in vec(i, j)]
                out = list(g2a[i, j])
                for k in nb[i]:
                    hk = [x / norm(vec(i, k)) for x in vec(i, k)]
                    a = w[k] / Z * sum(hj[t] * hk[t] for t in range(3))
                    for c in range(32):
                        out[c] += a * V[k][c]
                g2b[i, j] = out
        g1n = {}
        for i in range(N):
            T = [[0.0] * 4 for _ in range(32)]
            cc = [0.0] * 32
            for j in nb[i]:
                v = vec(i, j)
                r = norm(v)
                s = sw(r) / r
                R = [s] + [s * x / r for x in v]
                for c in range(32):
                    for a in range(4):
                        T[c][a] += g2b[i, j][c] * R[a] / m.sel
                    cc[c] += sw(r) * g2b[i, j][c] * g1[j][c] / m.sel
            D = [sum(T[c][a] * T[b][a] for a in range(4)) for c in range(32) for b in range(4)]
            x = g1[i] + D + cc
            g1n[i] = [g1[i][c] + math.tanh(z) for c, z in enumerate(lin(x, p[f"W1{l}"], p[f"b1{l}"]))]
        g1, g2 = g1n, g2b
    out = []
    for i in range(N):
        y1 = [math.tanh(z) for z in lin(g1[i], p["G1"], p["d1"])]
        y2 = [math.tanh(z) + y1[c] for c, z in enumerate(lin(y1, p["G2"], p["d2"]))]
        out.append(lin(y2, p["G3"], p["d3"])[0])
    return out


def test_scalar_loop_reevaluation(rm):
    X, t = _cluster(6, 21, spread=2.5, dmin=1.0)
    ref = np.array(_scalar_energies(rm, X.tolist(), t.tolist()))
    Ei = forward(rm, build_edges(rm, X, t, None))
    assert np.abs(Ei - ref).max() < 1e-9 * np.abs(ref).max()


def test_rotation_invariance(rm):
    X, t = _cluster(25, 5, spread=4.0)
    q = np.random.default_rng(8).normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    R = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                  [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                  [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])
    a = evaluate(rm, X, t, None)
    b = evaluate(rm, X @ R.T, t, None)
    assert abs(a["E"] - b["E"]) < 1e-9 * abs(a["E"])
    assert np.abs(a["F"] @ R.T - b["F"]).max() < 1e-8


def test_translation_and_permutation(rm, water192):
    s = water192
    a = evaluate(rm, s.coords, s.types, s.box)
    b = evaluate(rm, s.coords + np.array([3.3, -7.1, 20.0]), s.types, s.box)
    assert abs(a["E"] - b["E"]) < 1e-9 * abs(a["E"])
    perm = np.random.default_rng(2).permutation(s.natoms)
    c = evaluate(rm, s.coords[perm], s.types[perm], s.box)
    assert abs(a["E"] - c["E"]) < 1e-9 * abs(a["E"])
    assert np.abs(a["F"][perm] - c["F"]).max() < 1e-8


def test_receptive_field_is_three_hops(rm):
    X = np.array([[4.2 * k, 0.0, 0.0] for k in range(7)])
    t = np.array([0, 1, 2, 3, 4, 0, 1], dtype=np.int32)
    E0 = forward(rm, build_edges(rm, X, t, None))
    X1 = X.copy()
    X1[0] += np.array([0.3, 0.2, -0.1])
    E1 = forward(rm, build_edges(rm, X1, t, None))
    assert abs(E1[3] - E0[3]) > 1000 * np.spacing(abs(E0[3]))
    assert np.array_equal(E1[4:], E0[4:])


def test_smooth_through_cutoff(rm):
    X = np.array([[0.0, 0.0, 0.0], [1.0, 0.5, 0.0], [-0.8, 0.9, 0.3], [5.9, 0.0, 0.0]])
    t = np.array([0, 1, 2, 3], dtype=np.int32)
    Es = []
    for rr in np.arange(5.98, 6.02, 0.001):
        Y = X.copy()
        Y[3, 0] = rr
        Es.append(energy(rm, Y, t, None))
    assert np.abs(np.diff(np.diff(Es))).max() < 1e-6


def test_last_layer_norm(rm):
    """||G3||_2 of the seeded model, the constant of the GPU paths' energy bounds."""
    from tolerances import REP_G3NORM
    assert abs(np.linalg.norm(rm.p["G3"]) - REP_G3NORM) < 0.05
