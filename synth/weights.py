"""Seeded random-init model parameters and the binary model file.

The model is an attention-based deep potential of the DPA family (the paper's
Section II names its parts: a type-embedded per-neighbour embedding net, self
attention layers that update the representation residually, and a fitting net
giving per-atom energies).  Its sizes are fixed by ``ModelSpec``.  Trained
weights are not available, so the parameters are random draws from a seeded
PCG64 generator:

* weights of the embedding and fitting nets ~ N(0, 1/(fan_in + fan_out));
* every bias ~ N(0, 1); the type-embedding table ~ N(0, 1);
* attention projections W_Q, W_K, W_V, W_O ~ N(0, 1/fan_in);
* layer-norm gain 1, shift 0; per-type energy bias 0;
* the last fitting layer (weights and bias) is multiplied once by
  ``FORCE_SCALE`` so that forces on the 192-atom water box have an RMS of
  about 1 eV/A, which makes absolute force tolerances relative ones.

Model file layout (little endian), written here and read independently by
the oracle and by the HIP library:

====== ======= ==================================================
offset type    field
====== ======= ==================================================
0      8 bytes magic ``DPAMDv01``
8      16 i32  version, ntypes, tebd, e1, e2, M, n_attn, d_attn,
               M2, fit_hidden, n_fit_hidden, sel, nheads (0 or 1:
               one fitting net), 3 x reserved
72     4 f64   rc, rcs, ln_eps, force_scale
104    u64     seed
112    16      reserved (zero)
128    f64[]   arrays, in ``ModelSpec.array_shapes()`` order
====== ======= ==================================================

A model with nheads > 1 fitting nets (one descriptor shared by several fitting
heads, as the paper's multi-task models share one descriptor between branches)
appends, for each head h = 1 .. nheads-1, that head's fitting layers and energy
bias in the same order and shapes as head 0's (``ModelSpec.head_shapes``).  The
extra heads are drawn after every array of the single-head model, so head 0 and
everything before it are the same numbers as in the single-head file.
"""
from __future__ import annotations

import os
import struct
import tempfile
from dataclasses import dataclass

import numpy as np

MAGIC = b"DPAMDv01"
VERSION = 1
# Chosen with oracle/calibrate_force_scale.py so that the per-component force
# RMS of the 192-atom water box is 1 eV/A for seed 2602.
FORCE_SCALE = 2627.7633828759604


@dataclass(frozen=True)
class ModelSpec:
    ntypes: int = 5
    tebd: int = 8
    e1: int = 25
    e2: int = 50
    M: int = 100
    n_attn: int = 2
    d_attn: int = 128
    M2: int = 16
    fit_hidden: int = 240
    n_fit_hidden: int = 3
    sel: int = 120
    rc: float = 6.0
    rcs: float = 0.5
    ln_eps: float = 1e-5
    nheads: int = 1

    def fitting_shapes(self, prefix=""):
        fd = [self.M * self.M2] + [self.fit_hidden] * self.n_fit_hidden + [1]
        out = []
        for li in range(len(fd) - 1):
            out.append((f"{prefix}fit_W{li + 1}", (fd[li], fd[li + 1]), "glorot"))
            out.append((f"{prefix}fit_b{li + 1}", (fd[li + 1],), "unit"))
        out.append((f"{prefix}energy_bias", (self.ntypes,), "zero"))
        return out

    def head_shapes(self):
        """The arrays of the extra fitting heads 1 .. nheads-1, in file order."""
        out = []
        for h in range(1, self.nheads):
            out += self.fitting_shapes(f"head{h}_")
        return out

    def array_shapes(self):
        """(name, shape, kind) in file order; kind selects the init distribution."""
        out = [("type_embedding", (self.ntypes, self.tebd), "unit")]
        dims = [1 + 2 * self.tebd, self.e1, self.e2, self.M]
        for li in range(3):
            out.append((f"emb_W{li + 1}", (dims[li], dims[li + 1]), "glorot"))
            out.append((f"emb_b{li + 1}", (dims[li + 1],), "unit"))
        for a in range(self.n_attn):
            out.append((f"attn{a}_WQ", (self.M, self.d_attn), "fanin"))
            out.append((f"attn{a}_WK", (self.M, self.d_attn), "fanin"))
            out.append((f"attn{a}_WV", (self.M, self.d_attn), "fanin"))
            out.append((f"attn{a}_WO", (self.d_attn, self.M), "fanin"))
            out.append((f"attn{a}_gamma", (self.M,), "one"))
            out.append((f"attn{a}_beta", (self.M,), "zero"))
        return out + self.fitting_shapes()


def make_params(spec: ModelSpec = ModelSpec(), seed: int = 2602, force_scale: float | None = None):
    """Draw the parameters; returns an ordered dict name -> float64 array."""
    if force_scale is None:
        force_scale = FORCE_SCALE
    rng = np.random.default_rng(seed)
    params = {}
    for name, shape, kind in spec.array_shapes() + spec.head_shapes():
        if kind == "unit":
            a = rng.normal(0.0, 1.0, size=shape)
        elif kind == "glorot":
            a = rng.normal(0.0, np.sqrt(1.0 / (shape[0] + shape[1])), size=shape)
        elif kind == "fanin":
            a = rng.normal(0.0, np.sqrt(1.0 / shape[0]), size=shape)
        elif kind == "one":
            a = np.ones(shape)
        else:
            a = np.zeros(shape)
        params[name] = a.astype(np.float64)
    last = spec.n_fit_hidden + 1
    for h in range(spec.nheads):
        pre = f"head{h}_" if h else ""
        params[f"{pre}fit_W{last}"] *= force_scale
        params[f"{pre}fit_b{last}"] *= force_scale
    return params


def write_model_file(path: str, spec: ModelSpec = ModelSpec(), seed: int = 2602,
                     force_scale: float | None = None, params=None) -> str:
    if force_scale is None:
        force_scale = FORCE_SCALE
    if params is None:
        params = make_params(spec, seed, force_scale)
    ints = [VERSION, spec.ntypes, spec.tebd, spec.e1, spec.e2, spec.M, spec.n_attn, spec.d_attn,
            spec.M2, spec.fit_hidden, spec.n_fit_hidden, spec.sel, spec.nheads if spec.nheads > 1 else 0, 0, 0, 0]
    head = MAGIC + struct.pack("<16i", *ints)
    head += struct.pack("<4d", spec.rc, spec.rcs, spec.ln_eps, force_scale)
    head += struct.pack("<Q", seed) + bytes(16)
    assert len(head) == 128
    with open(path, "wb") as f:
        f.write(head)
        for name, shape, _ in spec.array_shapes() + spec.head_shapes():
            a = np.ascontiguousarray(params[name], dtype="<f8")
            assert a.shape == tuple(shape), (name, a.shape, shape)
            f.write(a.tobytes())
    return path


def default_model_file(seed: int = 2602, nheads: int = 1) -> str:
    """Write (once per process, seed and head count) the default model file to a temp dir
    and return its path.  nheads > 1: the same model with extra fitting heads."""
    d = os.path.join(tempfile.gettempdir(), f"dpamd_models_{os.getuid()}")
    os.makedirs(d, exist_ok=True)
    tag = f"_h{nheads}" if nheads > 1 else ""
    path = os.path.join(d, f"model_seed{seed}_fs{FORCE_SCALE!r}{tag}.bin")
    if not os.path.exists(path):
        tmp = path + f".{os.getpid()}.tmp"
        write_model_file(tmp, spec=ModelSpec(nheads=nheads), seed=seed)
        os.replace(tmp, path)
    return path
