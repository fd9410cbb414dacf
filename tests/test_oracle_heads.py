"""Pins of the oracle's multi-head fitting (several fitting nets on one descriptor), CPU only.

* Head 0 of a three-head model file is the single-head model: same arrays, same results.
* Head h's view uses the arrays the seeded generator drew for head h: an element-by-element
  scalar evaluation built from the generator's own arrays (not from the file reader) gives
  the same atomic energy.
* The forces of a weighted head combination are minus the gradient of the combined
  energy: central differences of sum_h w_h E^h at h = 1e-4 A.
"""
import numpy as np
import pytest

from oracle import load_model
from oracle.dp import evaluate, evaluate_heads, head_view, local_energy, atom_energy_and_grad
from oracle.neighbors import neighbor_list_cells
from scalar_model import atom_energy_scalar
from synth import config_system, default_model_file
from synth.weights import ModelSpec, make_params


@pytest.fixture(scope="module")
def m3():
    return load_model(default_model_file(nheads=3))


def test_head0_is_the_single_head_model(omodel, m3, water192, oracle_water192):
    s = water192
    r = evaluate(head_view(m3, 0), s.coords, s.types, s.box)
    assert r["E"] == oracle_water192["E"]
    assert np.array_equal(r["F"], oracle_water192["F"])


@pytest.mark.parametrize("h", [1, 2])
def test_head_view_uses_the_generated_head(m3, h):
    p = make_params(ModelSpec(nheads=3), seed=2602)
    v = head_view(m3, h)
    # a model object carrying the generator's arrays for head h, mapped to the oracle's names
    import copy
    g = copy.copy(v)
    g.p = dict(v.p)
    for li in range(1, 5):
        g.p[f"F{li}"] = p[f"head{h}_fit_W{li}"]
        g.p[f"c{li}"] = p[f"head{h}_fit_b{li}"]
    g.p["ebias"] = p[f"head{h}_energy_bias"]
    rng = np.random.default_rng(30 + h)
    dR = rng.normal(size=(3, 3))
    dR *= rng.uniform(1.0, 5.5, size=(3, 1)) / np.linalg.norm(dR, axis=1, keepdims=True)
    tj = np.array([0, 1, 3])
    Ev, _ = atom_energy_and_grad(v, 2, tj, dR, want_grad=False)
    Es = atom_energy_scalar(g, 2, tj.tolist(), dR.tolist())
    assert abs(Ev - Es) <= 1e-11 * abs(Es)
    E0, _ = atom_energy_and_grad(head_view(m3, 0), 2, tj, dR, want_grad=False)
    assert abs(Ev - E0) > 1e-3  # a different function


def test_combined_forces_are_the_gradient(m3, water192):
    s = water192
    w = np.array([0.25, -0.5, 1.25])
    r = evaluate_heads(m3, s.coords, s.types, s.box, w)
    nl, nn, _ = neighbor_list_cells(s.coords, s.box, m3.rc + 0.01, 400)
    rng = np.random.default_rng(12)
    hstep = 1e-4
    worst = 0.0
    for i in rng.choice(s.natoms, size=3, replace=False):
        atoms = [int(i)] + nl[i, :nn[i]].tolist()
        a = int(rng.integers(3))
        Xp = s.coords.copy(); Xp[i, a] += hstep
        Xm = s.coords.copy(); Xm[i, a] -= hstep
        ep = sum(w[h] * local_energy(head_view(m3, h), Xp, s.types, s.box, atoms) for h in range(3))
        em = sum(w[h] * local_energy(head_view(m3, h), Xm, s.types, s.box, atoms) for h in range(3))
        worst = max(worst, abs(-(ep - em) / (2 * hstep) - r["F"][i, a]))
    assert worst < 1e-6
    assert abs(r["E"] - float(np.dot(w, r["E_heads"]))) <= 1e-9 * abs(r["E"])
