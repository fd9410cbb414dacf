"""Pins of the oracle's model arithmetic against independent evaluations (CPU only)."""
import copy
import math

import mpmath
import numpy as np
import pytest

from oracle.dp import atom_energy_and_grad, evaluate, switch
from oracle.neighbors import neighbor_list_cells, min_image
from scalar_model import atom_energy_scalar


def _neigh(rng, n, rmin=0.9, rmax=5.9):
    v = rng.normal(size=(n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v * rng.uniform(rmin, rmax, size=(n, 1))


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (3, 2), (4, 3)])
def test_vectorised_equals_scalar_loops(omodel, n, seed):
    """The matrix form equals an element-by-element evaluation (catches transposes, index slips)."""
    rng = np.random.default_rng(seed)
    dR = _neigh(rng, n)
    tj = rng.integers(0, 5, size=n)
    ti = int(rng.integers(0, 5))
    Ev, _ = atom_energy_and_grad(omodel, ti, tj, dR, want_grad=False)
    Es = atom_energy_scalar(omodel, ti, [int(t) for t in tj], dR.tolist())
    assert abs(Ev - Es) <= 1e-11 * max(1.0, abs(Es))


def test_single_pair_high_precision(omodel):
    """N = 2, open boundary: one token per atom (P = 1, gate = 1); 50-digit evaluation of the same atom."""
    mpmath.mp.dps = 50
    dR = np.array([[1.3, -2.1, 0.7]])
    for ti, tj in ((0, 1), (2, 4)):
        Ev, _ = atom_energy_and_grad(omodel, ti, np.array([tj]), dR, want_grad=False)
        Emp = atom_energy_scalar(omodel, ti, [tj], dR.tolist(), num=mpmath.mpf, tanh=mpmath.tanh,
                                 exp=mpmath.exp, sqrt=mpmath.sqrt)
        assert abs(Ev - float(Emp)) <= 1e-13 * abs(float(Emp)) + 1e-12


def test_single_pair_force_matches_high_precision_derivative(omodel):
    mpmath.mp.dps = 40
    X = np.array([[0.0, 0.0, 0.0], [1.1, 2.3, -0.4]])
    t = np.array([0, 3])
    out = evaluate(omodel, X, t, None)
    u = X[1] / np.linalg.norm(X[1])

    def E_of_r(rr):
        d = [float(rr * mpmath.mpf(c)) for c in u]
        e0 = atom_energy_scalar(omodel, 0, [3], [d], num=mpmath.mpf, tanh=mpmath.tanh, exp=mpmath.exp,
                                sqrt=mpmath.sqrt)
        e1 = atom_energy_scalar(omodel, 3, [0], [[-c for c in d]], num=mpmath.mpf, tanh=mpmath.tanh,
                                exp=mpmath.exp, sqrt=mpmath.sqrt)
        return e0 + e1

    r0 = mpmath.mpf(float(np.linalg.norm(X[1])))
    h = mpmath.mpf("1e-7")
    dEdr = (E_of_r(r0 + h) - E_of_r(r0 - h)) / (2 * h)
    # force on atom 1 is -dE/dr along u
    assert np.allclose(out["F"][1], -float(dEdr) * u, atol=1e-9, rtol=1e-7)
    assert np.allclose(out["F"][0], -out["F"][1], atol=1e-12)


def _ln(x, eps):
    mu = x.mean(axis=1, keepdims=True)
    return (x - mu) / np.sqrt(((x - mu) ** 2).mean(axis=1, keepdims=True) + eps)


def _deeppot_se(m, t_i, t_j, dR):
    """Attention-free reference: environment, embedding, a LayerNorm per layer, descriptor and fitting."""
    p = m.p
    r = np.linalg.norm(dR, axis=1)
    sw, _ = switch(r, m.rc, m.rcs)
    s = sw / r
    R = np.column_stack([s, s[:, None] * dR / r[:, None]])
    z = np.column_stack([s, p["TE"][t_j], np.tile(p["TE"][t_i], (len(r), 1))])
    h1 = np.tanh(z @ p["W1"] + p["b1"])
    h2 = np.tanh(h1 @ p["W2"] + p["b2"]) + np.tile(h1, 2)
    G = np.tanh(h2 @ p["W3"] + p["b3"]) + np.tile(h2, 2)
    for _ in range(m.n_attn):           # Y = 0: each layer only normalises (gamma 1, beta 0)
        G = _ln(G, m.ln_eps)
    T = np.einsum("jm,jc->mc", G, R) / m.sel
    D = np.einsum("mc,ac->ma", T, T[:m.M2]).ravel()
    y = np.tanh(D @ p["F1"] + p["c1"])
    y = np.tanh(y @ p["F2"] + p["c2"]) + y
    y = np.tanh(y @ p["F3"] + p["c3"]) + y
    return float(y @ p["F4"][:, 0] + p["c4"][0] + p["ebias"][t_i])


def test_attention_off_reduces_to_deeppot_se(omodel):
    m = copy.deepcopy(omodel)
    for a in range(m.n_attn):
        m.p[f"WO{a}"] = np.zeros_like(m.p[f"WO{a}"])   # Y = 0 -> each layer is G <- LN(G)
    rng = np.random.default_rng(7)
    for n in (1, 5, 40):
        dR = _neigh(rng, n)
        tj = rng.integers(0, 5, size=n)
        E, _ = atom_energy_and_grad(m, 2, tj, dR, want_grad=False)
        assert abs(E - _deeppot_se(m, 2, tj, dR)) <= 1e-12 * max(1, abs(E))


def test_attention_changes_energy(omodel):
    """Guard against a silently inactive attention block."""
    m = copy.deepcopy(omodel)
    for a in range(m.n_attn):
        m.p[f"WO{a}"] = np.zeros_like(m.p[f"WO{a}"])
    rng = np.random.default_rng(8)
    dR = _neigh(rng, 12)
    tj = rng.integers(0, 5, size=12)
    E_on, _ = atom_energy_and_grad(omodel, 1, tj, dR, want_grad=False)
    E_off, _ = atom_energy_and_grad(m, 1, tj, dR, want_grad=False)
    assert abs(E_on - E_off) > 1e-3


def test_neighbour_beyond_cutoff_is_inert(omodel):
    """A token at r >= rc has sw = 0: it drops out of the softmax weights and of Rt."""
    rng = np.random.default_rng(9)
    dR = _neigh(rng, 6)
    tj = rng.integers(0, 5, size=6)
    E0, _ = atom_energy_and_grad(omodel, 0, tj, dR, want_grad=False)
    far = np.vstack([dR, [[0.0, 0.0, 6.0]]])
    E1, _ = atom_energy_and_grad(omodel, 0, np.append(tj, 1), far, want_grad=False)
    assert abs(E0 - E1) <= 1e-12 * abs(E0)


def test_energy_is_sum_of_atom_energies(omodel, oracle_water192):
    o = oracle_water192
    assert abs(o["E"] - math.fsum(o["E_i"].tolist())) == 0.0
    assert o["n_overflow"] == 0


def test_force_scale_gives_unit_rms(oracle_water192):
    rms = float(np.sqrt(np.mean(oracle_water192["F"] ** 2)))
    assert abs(rms - 1.0) < 1e-9


def test_last_layer_norm(omodel):
    """The constant the energy bounds are derived from: ||F4||_2 of the seeded model."""
    from tolerances import F4NORM
    assert abs(np.linalg.norm(omodel.p["F4"]) - F4NORM) < 1.0
