"""Seeded random-init parameters and the model file of the GNN-variant descriptor.

Sizes and parameter list are fixed by ``oracle.gnn.gnn_shapes``'s counterpart below
(node 64, edge 64, angle 32, three layers, fitting 64 -> 128 -> 128 -> 1).  Draws from
a seeded PCG64 generator: weights ~ N(0, 1/(fan_in + fan_out)), biases and the node
embedding ~ N(0, 1); the last fitting layer (G3, d3) is multiplied once by
``GNN_FORCE_SCALE`` so that forces on the 192-atom water box have an RMS of about
1 eV/A.

File layout (little endian): magic ``DPGNNv01``; 16 int32: version, ntypes, node,
edge, angle, layers, fit width, sel, asel, 7 x reserved; 4 float64: rc, rcs, rca,
force_scale; uint64 seed; 16 reserved bytes (128 bytes in all); then the float64
arrays in ``gnn_shapes`` order.
"""
from __future__ import annotations

import os
import struct
import tempfile

import numpy as np

MAGIC = b"DPGNNv01"
ND, ED, AD, NL, FH = 64, 64, 32, 3, 128
# 1 / (the force RMS of the unscaled model on the 192-atom water box), from oracle/gnn.py
GNN_FORCE_SCALE = 195.8985657080885


def gnn_shapes(ntypes: int = 5):
    """(name, shape, kind) of every parameter, in generation and file order."""
    out = [("TN", (ntypes, ND), "unit"), ("We0", (1, ED), "glorot"), ("be0", (ED,), "unit"),
           ("Wa0", (1, AD), "glorot"), ("ba0", (AD,), "unit")]
    for l in range(NL):
        out += [(f"Waa{l}", (AD + 64, AD), "glorot"), (f"baa{l}", (AD,), "unit"),
                (f"Wea{l}", (AD + 32, ED), "glorot"), (f"bea{l}", (ED,), "unit"),
                (f"Wee{l}", (2 * ND + ED, ED), "glorot"), (f"bee{l}", (ED,), "unit"),
                (f"Wnn{l}", (ND + ED, ND), "glorot"), (f"bnn{l}", (ND,), "unit")]
    out += [("G1", (ND, FH), "glorot"), ("d1", (FH,), "unit"), ("G2", (FH, FH), "glorot"), ("d2", (FH,), "unit"),
            ("G3", (FH, 1), "glorot"), ("d3", (1,), "unit")]
    return out


def make_gnn_params(seed: int = 3602, force_scale: float | None = None, ntypes: int = 5):
    if force_scale is None:
        force_scale = GNN_FORCE_SCALE
    rng = np.random.default_rng(seed)
    out = {}
    for name, shape, kind in gnn_shapes(ntypes):
        if kind == "unit":
            a = rng.normal(0.0, 1.0, size=shape)
        else:
            a = rng.normal(0.0, np.sqrt(1.0 / (shape[0] + shape[1])), size=shape)
        out[name] = a.astype(np.float64)
    out["G3"] *= force_scale
    out["d3"] *= force_scale
    return out


def write_gnn_file(path: str, seed: int = 3602, force_scale: float | None = None, params=None,
                   rc=6.0, rcs=0.5, rca=4.0, sel=120, asel=48, ntypes=5) -> str:
    if force_scale is None:
        force_scale = GNN_FORCE_SCALE
    if params is None:
        params = make_gnn_params(seed, force_scale, ntypes)
    ints = [1, ntypes, ND, ED, AD, NL, FH, sel, asel, 0, 0, 0, 0, 0, 0, 0]
    head = MAGIC + struct.pack("<16i", *ints) + struct.pack("<4d", rc, rcs, rca, force_scale)
    head += struct.pack("<Q", seed) + bytes(16)
    assert len(head) == 128
    with open(path, "wb") as f:
        f.write(head)
        for name, shape, _ in gnn_shapes(ntypes):
            a = np.ascontiguousarray(params[name], dtype="<f8")
            assert a.shape == tuple(shape), name
            f.write(a.tobytes())
    return path


def default_gnn_file(seed: int = 3602) -> str:
    d = os.path.join(tempfile.gettempdir(), f"dpamd_models_{os.getuid()}")
    os.makedirs(d, exist_ok=True)
    path = os.path.join(d, f"gnn_seed{seed}_fs{GNN_FORCE_SCALE!r}.bin")
    if not os.path.exists(path):
        tmp = path + f".{os.getpid()}.tmp"
        write_gnn_file(tmp, seed=seed)
        os.replace(tmp, path)
    return path
