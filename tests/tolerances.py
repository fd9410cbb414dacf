"""Numeric acceptance bounds of the GPU paths against the FP64 oracle.

Forces are scaled so that their RMS on the 192-atom water box is 1 eV/A, so
absolute force bounds are also relative ones.  Atomic energies are then
O(1e3) eV (the same scale multiplies the last fitting layer), so energy bounds
are stated relative to the oracle's energies:
  e_atom_rel = max_i |dE_i| / max_i |E_i|,   e_rel = |dE| / |E|.

FP32 path: force RMSE <= 1e-5 eV/A (the stated target), max 1e-4.  E_i is a
240-term dot product of O(1) activations with O(100) weights; float32
rounding of the activations (2^-24 relative) over ~sqrt(240) terms gives
~1e-6 of |E_i|: bounds 5e-6 (per atom) and 2e-6 (total).  The virial is a
float64 sum of float32 pair terms: 1e-5 of its largest component.

BF16 path: the embedding and attention products take bfloat16 operands (2^-9
relative rounding per operand); the fitting net splits each operand into two
bfloat16 terms (three products, ~2^-17), so the energy error comes from the
descriptor.  One rounding of G (O(1) entries) per product moves D by ~2^-9 /
sqrt(#terms) relative and E_i by ~1e-5 of |E_i|; forces are differences of
pair terms of O(1) eV/A carrying ~2^-9 relative error each.  Measured on the
water box, the 1k-atom chain and an open cluster: force RMSE 2.7e-3 eV/A, max
1.2e-2, E_i 3.2e-5, E 9.4e-6, virial 3.4e-3 (relative).  The bounds are those
figures with a margin of 2-3x: forces 6e-3 RMSE and 4e-2 max, E_i 1e-4, E 5e-5,
virial 1e-2.
"""
FP32 = dict(f_rmse=1e-5, f_max=1e-4, e_atom_rel=5e-6, e_rel=2e-6, vir_rel=1e-5)
BF16 = dict(f_rmse=6e-3, f_max=4e-2, e_atom_rel=1e-4, e_rel=5e-5, vir_rel=1e-2)
TOL = {"fp32": FP32, "bf16": BF16}


def compare(gpu, ref, n):
    import numpy as np
    dF = gpu["F"] - ref["F"]
    out = dict(
        f_rmse=float(np.sqrt(np.mean(dF ** 2))),
        f_max=float(np.max(np.abs(dF))),
        e_per_atom=abs(gpu["E"] - ref["E"]) / n,
        e_rel=abs(gpu["E"] - ref["E"]) / abs(ref["E"]),
        vir_rel=float(np.max(np.abs(gpu["virial"] - ref["virial"])) / max(1e-30, np.max(np.abs(ref["virial"])))),
    )
    if "E_i" in gpu and "E_i" in ref:
        out["e_atom_rel"] = float(np.max(np.abs(gpu["E_i"] - ref["E_i"])) / np.max(np.abs(ref["E_i"])))
    return out


def assert_within(metrics, prec):
    tol = TOL[prec]
    bad = {k: (v, tol[k]) for k, v in metrics.items() if k in tol and not v <= tol[k]}
    assert not bad, f"{prec}: outside tolerance {bad}; all metrics {metrics}"
