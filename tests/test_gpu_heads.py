"""Several fitting heads on one descriptor (GPU vs the FP64 oracle).

A three-head model file: head 0 is the single-head model, heads 1 and 2 are further
seeded fitting nets.  The library evaluates the descriptor once and every head on it,
and returns E = sum_h w_h E^h with its forces and virial; each head's own energy is
read back as well.
"""
import numpy as np
import pytest

from oracle import load_model
from oracle.dp import evaluate, evaluate_heads, head_view
from synth import config_system, default_model_file
from tolerances import TOL, compare, assert_within

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def m3_path():
    return default_model_file(nheads=3)


@pytest.fixture(scope="module")
def om3(m3_path):
    return load_model(m3_path)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_default_weights_equal_single_head_model(gpu_models, m3_path, water192, prec):
    from paper_2602_02234_amd import Model
    s = water192
    m = Model(m3_path, prec)
    assert m.nheads == 3
    a = m.compute(s.coords, s.types, s.box, atom_energy=True)
    b = gpu_models[prec].compute(s.coords, s.types, s.box, atom_energy=True)
    assert a["E"] == b["E"] and np.array_equal(a["F"], b["F"]) and np.array_equal(a["virial"], b["virial"])
    m.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_each_head_and_a_combination_match_oracle(m3_path, om3, prec):
    from paper_2602_02234_amd import Model
    s = config_system("chain1k")
    m = Model(m3_path, prec)
    for h in range(3):
        w = np.zeros(3)
        w[h] = 1.0
        m.set_head_weights(w)
        out = m.compute(s.coords, s.types, s.box, atom_energy=True)
        ref = evaluate(head_view(om3, h), s.coords, s.types, s.box)
        met = compare(out, ref, s.natoms)
        print(prec, "head", h, met)
        assert_within(met, prec)
    w = np.array([0.25, -0.5, 1.25])
    m.set_head_weights(w)
    out = m.compute(s.coords, s.types, s.box, atom_energy=True)
    ref = evaluate_heads(om3, s.coords, s.types, s.box, w)
    met = compare(out, ref, s.natoms)
    print(prec, "combination", met)
    assert_within(met, prec)
    Eh = m.head_energies()[0]
    assert np.all(np.abs(Eh - ref["E_heads"]) / s.natoms <= TOL[prec]["e_per_atom"]), (Eh, ref["E_heads"])
    m.close()


def test_head_weights_apply_to_graph_replays(m3_path):
    """Weights are kernel arguments: changing them must not replay a graph captured before."""
    import torch
    from paper_2602_02234_amd import Model
    s = config_system("water192")
    m, ref = Model(m3_path, "bf16"), Model(m3_path, "bf16")
    m.set_graph(True)
    dev = torch.device("cuda:0")
    X, T = torch.tensor(s.coords, device=dev), torch.tensor(s.types, device=dev)
    F = torch.zeros((s.natoms, 3), dtype=torch.float64, device=dev)
    E = torch.zeros(1, dtype=torch.float64, device=dev)
    for w in ([1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.5, 0.0, 0.5]):
        m.set_head_weights(w)
        ref.set_head_weights(w)
        m.compute_device(X, T, s.box, forces=F, energy=E)
        torch.cuda.synchronize()
        r = ref.compute(s.coords, s.types, s.box)
        assert E.item() == r["E"] and np.array_equal(F.cpu().numpy(), r["F"]), w
    m.close()
    ref.close()
