"""Seeded random-init parameters and the model file of the repformer-style model.

Sizes (pair width 32, node width 64, axis columns 4, three layers, fitting
64 -> 128 -> 128 -> 1) and the parameter list are fixed by ``rep_shapes`` below.
Draws from a seeded PCG64 generator: weights ~ N(0, 1/(fan_in + fan_out)), biases and
the node embedding ~ N(0, 1); the last fitting layer (G3, d3) is multiplied once by
``REP_FORCE_SCALE`` so that forces on the 192-atom water box have an RMS of about
1 eV/A.

File layout (little endian): magic ``DPREPv01``; 16 int32: version, ntypes, node
width, pair width, axis columns, layers, fit width, sel, 8 x reserved; 3 float64: rc,
rcs, force_scale; uint64 seed; 24 reserved bytes (128 bytes in all); then the float64
arrays in ``rep_shapes`` order.
"""
from __future__ import annotations

import os
import struct
import tempfile

import numpy as np

MAGIC = b"DPREPv01"
G1D, G2D, NAX, NL, FH = 64, 32, 4, 3, 128
XD = G1D + G2D * NAX + G2D
# 1 / (the force RMS of the unscaled model on the 192-atom water box), from oracle/repformer.py
REP_FORCE_SCALE = 666.3744038611736


def rep_shapes(ntypes: int = 5):
    """(name, shape, kind) of every parameter, in generation and file order."""
    out = [("TN", (ntypes, G1D), "unit"), ("Wp0", (1, G2D), "glorot"), ("bp0", (G2D,), "unit")]
    for l in range(NL):
        out += [(f"Wa{l}", (G2D + G1D, G2D), "glorot"), (f"ba{l}", (G2D,), "unit"),
                (f"Wq{l}", (G2D, G2D), "glorot"), (f"Wk{l}", (G2D, G2D), "glorot"), (f"Wv{l}", (G2D, G2D), "glorot"),
                (f"W1{l}", (XD, G1D), "glorot"), (f"b1{l}", (G1D,), "unit")]
    out += [("G1", (G1D, FH), "glorot"), ("d1", (FH,), "unit"), ("G2", (FH, FH), "glorot"), ("d2", (FH,), "unit"),
            ("G3", (FH, 1), "glorot"), ("d3", (1,), "unit")]
    return out


def make_rep_params(seed: int = 4602, force_scale: float | None = None, ntypes: int = 5):
    if force_scale is None:
        force_scale = REP_FORCE_SCALE
    rng = np.random.default_rng(seed)
    out = {}
    for name, shape, kind in rep_shapes(ntypes):
        if kind == "unit":
            a = rng.normal(0.0, 1.0, size=shape)
        else:
            a = rng.normal(0.0, np.sqrt(1.0 / (shape[0] + shape[1])), size=shape)
        out[name] = a.astype(np.float64)
    out["G3"] *= force_scale
    out["d3"] *= force_scale
    return out


def write_rep_file(path: str, seed: int = 4602, force_scale: float | None = None, params=None,
                   rc=6.0, rcs=0.5, sel=120, ntypes=5) -> str:
    if force_scale is None:
        force_scale = REP_FORCE_SCALE
    if params is None:
        params = make_rep_params(seed, force_scale, ntypes)
    ints = [1, ntypes, G1D, G2D, NAX, NL, FH, sel, 0, 0, 0, 0, 0, 0, 0, 0]
    head = MAGIC + struct.pack("<16i", *ints) + struct.pack("<3d", rc, rcs, force_scale)
    head += struct.pack("<Q", seed) + bytes(24)
    assert len(head) == 128
    with open(path, "wb") as f:
        f.write(head)
        for name, shape, _ in rep_shapes(ntypes):
            a = np.ascontiguousarray(params[name], dtype="<f8")
            assert a.shape == tuple(shape), name
            f.write(a.tobytes())
    return path


def default_rep_file(seed: int = 4602) -> str:
    d = os.path.join(tempfile.gettempdir(), f"dpamd_models_{os.getuid()}")
    os.makedirs(d, exist_ok=True)
    path = os.path.join(d, f"rep_seed{seed}_fs{REP_FORCE_SCALE!r}.bin")
    if not os.path.exists(path):
        tmp = path + f".{os.getpid()}.tmp"
        write_rep_file(tmp, seed=seed)
        os.replace(tmp, path)
    return path
