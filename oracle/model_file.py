"""Reader of the model file (oracle side; the library has its own C++ reader).

Layout: a 128-byte little-endian header (magic ``DPAMDv01``; 16 int32:
version, ntypes, tebd, e1, e2, M, n_attn, d_attn, M2, fit_hidden,
n_fit_hidden, sel, 4 reserved; 4 float64: rc, rcs, ln_eps, force_scale;
uint64 seed; 16 reserved bytes) followed by float64 arrays in this order:
type embedding [ntypes][tebd]; embedding layers (W [in][out], b [out]) for
17->e1->e2->M; per attention layer WQ, WK, WV [M][d], WO [d][M], gamma, beta
[M]; fitting layers (W [in][out], b [out]) for M*M2 -> H -> ... -> 1; per-type
energy bias [ntypes].  The first reserved int is the number of fitting heads
(0 or 1: one); a model with more appends, for each further head, its fitting
layers and energy bias in the same order (``Model.heads[h]``, head 0 being the
arrays above).
"""
from __future__ import annotations

import struct
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Model:
    ntypes: int
    tebd: int
    e1: int
    e2: int
    M: int
    n_attn: int
    d_attn: int
    M2: int
    fit_hidden: int
    n_fit_hidden: int
    sel: int
    rc: float
    rcs: float
    ln_eps: float
    force_scale: float
    seed: int
    p: dict = field(default_factory=dict)
    heads: list = field(default_factory=list)  # per head: {"F1", "c1", ..., "F4", "c4", "ebias"}


def load_model(path: str) -> Model:
    with open(path, "rb") as f:
        raw = f.read()
    if raw[:8] != b"DPAMDv01":
        raise ValueError("not a model file")
    ints = struct.unpack_from("<16i", raw, 8)
    version, ntypes, tebd, e1, e2, M, n_attn, d_attn, M2, H, nfh, sel, nheads = ints[:13]
    nheads = max(1, nheads)
    if version != 1:
        raise ValueError(f"unsupported model file version {version}")
    rc, rcs, eps, fscale = struct.unpack_from("<4d", raw, 72)
    (seed,) = struct.unpack_from("<Q", raw, 104)
    m = Model(ntypes, tebd, e1, e2, M, n_attn, d_attn, M2, H, nfh, sel, rc, rcs, eps, fscale, seed)
    off = 128

    def take(name, *shape, into=None):
        nonlocal off
        n = int(np.prod(shape))
        a = np.frombuffer(raw, dtype="<f8", count=n, offset=off).reshape(shape).astype(np.float64)
        off += 8 * n
        (m.p if into is None else into)[name] = a

    take("TE", ntypes, tebd)
    dims = [1 + 2 * tebd, e1, e2, M]
    for li in range(3):
        take(f"W{li + 1}", dims[li], dims[li + 1])
        take(f"b{li + 1}", dims[li + 1])
    for a in range(n_attn):
        take(f"WQ{a}", M, d_attn)
        take(f"WK{a}", M, d_attn)
        take(f"WV{a}", M, d_attn)
        take(f"WO{a}", d_attn, M)
        take(f"gamma{a}", M)
        take(f"beta{a}", M)
    fd = [M * M2] + [H] * nfh + [1]
    for h in range(nheads):
        d = m.p if h == 0 else {}
        for li in range(len(fd) - 1):
            take(f"F{li + 1}", fd[li], fd[li + 1], into=d)
            take(f"c{li + 1}", fd[li + 1], into=d)
        take("ebias", ntypes, into=d)
        m.heads.append({k: d[k] for k in [f"F{li + 1}" for li in range(len(fd) - 1)] +
                        [f"c{li + 1}" for li in range(len(fd) - 1)] + ["ebias"]})
    if off != len(raw):
        raise ValueError(f"model file size mismatch: parsed {off} of {len(raw)} bytes")
    return m
