"""Numeric acceptance bounds of the GPU paths against the FP64 oracle.

Forces are scaled so that their RMS on the 192-atom water box is 1 eV/A (the
last fitting layer F4, c4 carries that scale), so absolute force bounds are also
relative ones.  Energies are bounded in absolute eV, per atom:

  e_atom  = max_i |dE_i|          (eV)
  e_per_atom = |dE| / N           (eV/atom)

Derivation.  E_i = y3 . F4 + c4 + ebias[t_i].  Both paths sum that last layer in
float64 with float64 F4, c4 and ebias, so the energy error is the error of the
240 activations y3 (|y3| <= 3) carried to E_i by F4: sum_k F4_k dy3_k, of size
c u ||F4||_2, where u is the path's unit roundoff and ||F4||_2 = 2734 eV for the
seeded model (the constant F4NORM below, pinned by
tests/test_oracle_model.py::test_last_layer_norm).  c counts the roundings that
reach y3, relative to |y3|: those of the fitting net itself and those of every
float32 step upstream (environment, two attention layers with softmax and
LayerNorm, T, D), amplified by the fitting net's sensitivity to D.

* FP32 (u = 2^-24, u ||F4|| = 1.6e-4 eV): measured c up to 8.5 per atom (max
  |dE_i| 1.4e-3 eV) and up to 1.4 for |dE|/N (water box, 1k chain, open and
  dense clusters, 10k-40k chains).  Bounds c = 16 per atom, c = 4 for |dE|/N (the
  errors of alike atoms are correlated, so the mean does not shrink as 1/sqrt(N)).
* BF16 (u = 2^-8, u ||F4|| = 10.7 eV): the descriptor products round their
  operands to bfloat16; the fitting net (split bfloat16 operands, ~2^-16) passes
  the descriptor's error through.  That error is averaged over the ~90 neighbour
  rows of T and the 1600 features of D, so c is far below 1: measured up to 2.2e-3
  per atom and 1.1e-3 for |dE|/N.  Bounds c = 6e-3 and 2e-3.

Clusters denser than water (forces of RMS s > 1 eV/A) are compared after dividing
forces and energies by s, since every error above grows with the size of the
descriptor, as the forces do.

The survey's contract (FP32 1e-6 eV/atom, BF16 2e-3 eV/atom) assumed an O(1)
energy scale.  Scaling the last layer by 2628 so that forces have RMS 1 eV/A makes
u ||F4|| = 1.6e-4 eV, so no float32 network meets 1e-6 eV/atom at this force
scale; the measured values are reported beside the bounds.

Forces: FP32 RMSE <= 1e-5 eV/A (the stated target), max 1e-4.  BF16: the pair
terms of O(1) eV/A carry ~u_bf16 relative error each; measured RMSE 2.7e-3, max
1.2e-2 on the water box, the 1k chain and an open cluster; bounds 6e-3 and 4e-2.
Virial (relative to its largest component): a float64 sum of float32 pair terms,
1e-5 (FP32); 1e-2 (BF16, measured 3.4e-3).
"""
U32 = 2.0 ** -24
UBF16 = 2.0 ** -8
F4NORM = 2734.0  # ||F4||_2 of the seeded model file, eV

FP32 = dict(f_rmse=1e-5, f_max=1e-4, e_atom=16 * U32 * F4NORM, e_per_atom=4 * U32 * F4NORM, vir_rel=1e-5)
BF16 = dict(f_rmse=6e-3, f_max=4e-2, e_atom=6e-3 * UBF16 * F4NORM, e_per_atom=2e-3 * UBF16 * F4NORM,
            vir_rel=1e-2)
TOL = {"fp32": FP32, "bf16": BF16}


def compare(gpu, ref, n, scale=1.0):
    """Error metrics of a GPU result against the oracle's; forces and energies divided
    by `scale` (the oracle's force RMS for clusters denser than water, else 1)."""
    import numpy as np
    dF = (gpu["F"] - ref["F"]) / scale
    out = dict(
        f_rmse=float(np.sqrt(np.mean(dF ** 2))),
        f_max=float(np.max(np.abs(dF))),
        e_per_atom=abs(gpu["E"] - ref["E"]) / n / scale,
        vir_rel=float(np.max(np.abs(gpu["virial"] - ref["virial"])) / max(1e-30, np.max(np.abs(ref["virial"])))),
    )
    if "E_i" in gpu and "E_i" in ref:
        out["e_atom"] = float(np.max(np.abs(gpu["E_i"] - ref["E_i"]))) / scale
    return out


def assert_within(metrics, prec):
    tol = TOL[prec]
    bad = {k: (v, tol[k]) for k, v in metrics.items() if k in tol and not v <= tol[k]}
    assert not bad, f"{prec}: outside tolerance {bad}; all metrics {metrics}"


# ---------------------------------------------------------------- GNN variant
# The same reasoning with the GNN model's last layer: E_i = y2 . G3 + d3 is summed in
# float64 from float32 y2 (|y2| <= 2), so the energy error is c u ||G3||_2 with
# ||G3||_2 = 187.9 eV for the seeded model (G3NORM, pinned by
# tests/test_oracle_gnn.py::test_last_layer_norm).  Its forces are scaled to RMS 1 eV/A
# on the water box as well.  Measured on the water box, a 60-atom open cluster, the 1k
# chain and sampled atoms of the 40k chain:
# * FP32: c = 9.8 per atom (1.1e-4 eV), 0.37 for |dE|/N; force RMSE 5.4e-7, max
#   2.4e-6; virial 4e-8.  Bounds c = 16 and 4, forces 1e-5 / 1e-4, virial 1e-5.
# * BF16 (the angle-row and edge-row products on bfloat16 operands, three layers deep;
#   the per-edge and per-atom bias terms in float32): c = 0.024 per atom (0.018 eV),
#   0.011 for |dE|/N (a systematic offset of about -0.008 eV per atom, the same sign on
#   every system); force RMSE 9.2e-4, max 4.0e-3; virial 6.7e-4.  Bounds c = 0.08 and
#   0.02, forces 2e-3 / 1e-2, virial 2e-3.
G3NORM = 187.9
GNN_FP32 = dict(f_rmse=1e-5, f_max=1e-4, e_atom=16 * U32 * G3NORM, e_per_atom=4 * U32 * G3NORM, vir_rel=1e-5)
GNN_BF16 = dict(f_rmse=2e-3, f_max=1e-2, e_atom=0.08 * UBF16 * G3NORM, e_per_atom=0.02 * UBF16 * G3NORM,
                vir_rel=2e-3)
TOL_GNN = {"fp32": GNN_FP32, "bf16": GNN_BF16}


def assert_within_gnn(metrics, prec):
    tol = TOL_GNN[prec]
    bad = {k: (v, tol[k]) for k, v in metrics.items() if k in tol and not v <= tol[k]}
    assert not bad, f"GNN {prec}: outside tolerance {bad}; all metrics {metrics}"


# ---------------------------------------------------------------- repformer-style model
# E_i = y2 . G3 + d3 in float64 from float32 y2; ||G3||_2 = 620.3 eV for the seeded
# model (REP_G3NORM, pinned by tests/test_oracle_repformer.py::test_last_layer_norm).
REP_G3NORM = 620.3
REP_FP32 = dict(f_rmse=1e-5, f_max=1e-4, e_atom=16 * U32 * REP_G3NORM, e_per_atom=4 * U32 * REP_G3NORM, vir_rel=1e-5)
TOL_REP = {"fp32": REP_FP32}
