"""A DPA2-style repformer model in plain float64 NumPy, with a hand-written gradient --
TEST INFRASTRUCTURE ONLY (imported by tests and the smoke check, never by the library).

The paper's DPA2 models (Section II) stack repformer layers that update a single-atom
representation g1 and a pair representation g2 and pass messages from neighbour to
neighbour, so the receptive field grows by rc per layer; the paper names the parts
only.  This is the reading used here:

Environment as in the attention model: Delta_ij = x_j - x_i, r, sw(r) (quintic, smooth
from rcs = 0.5 A to rc = 6 A), s = sw / r, rhat = Delta / r, R_ij = (s, s rhat).

Features: g1_i (64) per atom, g2_ij (32) per edge (j in N(i), the rc lists):
    g1_i = TN[t_i];   g2_ij = tanh(s_ij Wp0 + bp0)
Three layers l = 0, 1, 2:
    pair update from the neighbour:   g2_ij <- g2_ij + tanh([g2_ij, g1_j] Wa_l + ba_l)
    gated self-attention over the neighbours of i (one head, width 32, no biases):
        Q, K, V = g2 Wq_l, g2 Wk_l, g2 Wv_l;   S_jk = Q_j . K_k / sqrt(32)
        P_jk = sw_k exp(S_jk) / sum_k' sw_k' exp(S_jk');   A_jk = P_jk (rhat_j . rhat_k)
        g2_ij <- g2_ij + sum_k A_jk V_k
    node update:  T_i = sum_j g2_ij R_ij^T / sel (32 x 4);  D_i = T_i T_i[:4]^T (32 x 4,
        flattened row-major);  c_i = sum_j sw_ij g2_ij * g1_j[:32] / sel;
        g1_i <- g1_i + tanh([g1_i, D_i, c_i] W1_l + b1_l)      (64 + 128 + 32 -> 64)
Energy:  y1 = tanh(g1 G1 + d1);  y2 = tanh(y1 G2 + d2) + y1;  E_i = y2 G3 + d3.

The layer's pair update and convolution read the neighbours' g1 of the layer before,
so E_i depends on atoms up to 3 rc away.  Every term a neighbour adds to g1 or to the
attention carries R or its switch, so E is smooth as atoms cross rc.

Gradient.  E depends on the positions only through Delta_ij, so g_ij = dE/dDelta_ij
(E the total energy) gives F_i = sum_j g_ij - sum_j g_ji and the virial, as for the
other models.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from .dp import switch
from .neighbors import neighbor_list_cells, min_image, _box_lengths

G1D, G2D, NAX, NL = 64, 32, 4, 3  # node width, pair width, axis columns of D, layers
FH = 128
XD = G1D + G2D * NAX + G2D        # node-update input width (224)


@dataclass
class RepModel:
    ntypes: int = 5
    rc: float = 6.0
    rcs: float = 0.5
    sel: int = 120
    force_scale: float = 1.0
    p: dict = field(default_factory=dict)


def rep_shapes(ntypes):
    out = [("TN", (ntypes, G1D)), ("Wp0", (1, G2D)), ("bp0", (G2D,))]
    for l in range(NL):
        out += [(f"Wa{l}", (G2D + G1D, G2D)), (f"ba{l}", (G2D,)), (f"Wq{l}", (G2D, G2D)), (f"Wk{l}", (G2D, G2D)),
                (f"Wv{l}", (G2D, G2D)), (f"W1{l}", (XD, G1D)), (f"b1{l}", (G1D,))]
    out += [("G1", (G1D, FH)), ("d1", (FH,)), ("G2", (FH, FH)), ("d2", (FH,)), ("G3", (FH, 1)), ("d3", (1,))]
    return out


def load_rep_model(path: str) -> RepModel:
    """Reads a repformer model file (magic DPREPv01; layout in synth/rep_weights.py)."""
    import struct
    raw = open(path, "rb").read()
    if raw[:8] != b"DPREPv01":
        raise ValueError("not a repformer model file")
    iv = struct.unpack_from("<16i", raw, 8)
    version, ntypes, g1d, g2d, nax, nl, fh, sel = iv[:8]
    if version != 1 or (g1d, g2d, nax, nl, fh) != (G1D, G2D, NAX, NL, FH):
        raise ValueError("unsupported repformer model file")
    rc, rcs, fscale = struct.unpack_from("<3d", raw, 72)
    m = RepModel(ntypes=ntypes, rc=rc, rcs=rcs, sel=sel, force_scale=fscale)
    off = 128
    for name, shape in rep_shapes(ntypes):
        k = int(np.prod(shape))
        m.p[name] = np.frombuffer(raw, dtype="<f8", count=k, offset=off).reshape(shape).astype(np.float64)
        off += 8 * k
    if off != len(raw):
        raise ValueError("repformer model file size mismatch")
    return m


def build_edges(m: RepModel, X, types, box, nlist=None, nnei=None):
    """Edges (centre, neighbour, Delta) from the neighbour lists, grouped by centre in list order."""
    X = np.asarray(X, dtype=np.float64)
    L = _box_lengths(box)
    if nlist is None:
        nlist, nnei, _ = neighbor_list_cells(X, box, m.rc, m.sel)
    src = np.repeat(np.arange(X.shape[0]), nnei)
    dst = np.concatenate([nlist[i, :nnei[i]] for i in range(X.shape[0])]).astype(np.int64) if len(src) else \
        np.zeros(0, dtype=np.int64)
    D = min_image(X[dst] - X[src], L)
    start = np.concatenate([[0], np.cumsum(nnei)]).astype(np.int64)
    return dict(src=src, dst=dst, D=D, start=start, types=np.asarray(types), N=X.shape[0], nlist=nlist, nnei=nnei)


def _geometry(m, D):
    r = np.sqrt(np.sum(D * D, axis=1))
    sw, dsw = switch(r, m.rc, m.rcs)
    s = sw / r
    rh = D / r[:, None]
    R = np.concatenate([s[:, None], s[:, None] * rh], axis=1)
    return r, sw, dsw, s, rh, R


def _attention(Q, K, V, sw, rh):
    """One centre's gated attention output and the values its gradient needs."""
    S = Q @ K.T / math.sqrt(G2D)
    ex = np.exp(S - S.max(axis=1, keepdims=True))
    e = ex * sw[None, :]
    Z = e.sum(axis=1, keepdims=True)
    P = e / Z
    Gt = rh @ rh.T
    A = P * Gt
    return A @ V, dict(P=P, Gt=Gt, A=A, exZ=ex / Z)


# ----------------------------------------------------------------------------- forward
def forward(m: RepModel, g: dict, keep: bool = False):
    p = m.p
    src, dst, start = g["src"], g["dst"], g["start"]
    r, sw, dsw, s, rh, R = _geometry(m, g["D"])
    g1 = p["TN"][g["types"]]
    g2 = np.tanh(s[:, None] * p["Wp0"][0] + p["bp0"])
    tape = []
    for l in range(NL):
        xa = np.concatenate([g2, g1[dst]], axis=1)
        ta = np.tanh(xa @ p[f"Wa{l}"] + p[f"ba{l}"])
        g2a = g2 + ta
        Q, K, V = g2a @ p[f"Wq{l}"], g2a @ p[f"Wk{l}"], g2a @ p[f"Wv{l}"]
        Y = np.zeros_like(g2a)
        att = []
        for i in range(g["N"]):
            a, b = start[i], start[i + 1]
            if b == a:
                att.append(None)
                continue
            Y[a:b], rec = _attention(Q[a:b], K[a:b], V[a:b], sw[a:b], rh[a:b])
            att.append(rec)
        g2b = g2a + Y
        T = np.zeros((g["N"], G2D, 4))
        np.add.at(T, src, g2b[:, :, None] * R[:, None, :])
        T /= m.sel
        Dd = np.einsum("nma,nba->nmb", T, T[:, :NAX, :]).reshape(g["N"], G2D * NAX)
        c = np.zeros((g["N"], G2D))
        np.add.at(c, src, sw[:, None] * g2b * g1[dst, :G2D])
        c /= m.sel
        xn = np.concatenate([g1, Dd, c], axis=1)
        tn = np.tanh(xn @ p[f"W1{l}"] + p[f"b1{l}"])
        g1n = g1 + tn
        tape.append(dict(g1=g1, g2=g2, ta=ta, g2a=g2a, Q=Q, K=K, V=V, att=att, g2b=g2b, T=T, tn=tn))
        g1, g2 = g1n, g2b
    y1 = np.tanh(g1 @ p["G1"] + p["d1"])
    y2 = np.tanh(y1 @ p["G2"] + p["d2"]) + y1
    Ei = (y2 @ p["G3"])[:, 0] + p["d3"][0]
    if not keep:
        return Ei
    return Ei, dict(tape=tape, y1=y1, y2=y2, geo=(r, sw, dsw, s, rh, R))


# ----------------------------------------------------------------------------- gradient
def pair_gradients(m: RepModel, g: dict):
    """E_i and g_e = dE/dDelta_e for every edge e (E the total energy), reverse mode."""
    p = m.p
    src, dst, start = g["src"], g["dst"], g["start"]
    Ei, f = forward(m, g, keep=True)
    r, sw, dsw, s, rh, R = f["geo"]
    dy2 = np.broadcast_to(p["G3"][:, 0], f["y2"].shape).copy()
    t2 = f["y2"] - f["y1"]
    dy1 = (dy2 * (1.0 - t2 * t2)) @ p["G2"].T + dy2
    dg1 = (dy1 * (1.0 - f["y1"] ** 2)) @ p["G1"].T
    dg2 = np.zeros((len(src), G2D))
    dsw_acc = np.zeros(len(src))
    drh = np.zeros_like(rh)
    dR = np.zeros_like(R)
    for l in reversed(range(NL)):
        t = f["tape"][l]
        g1, g2b = t["g1"], t["g2b"]
        # node update
        dz = dg1 * (1.0 - t["tn"] ** 2)
        dxn = dz @ p[f"W1{l}"].T
        dg1_in = dg1 + dxn[:, :G1D]
        dD = dxn[:, G1D:G1D + G2D * NAX].reshape(-1, G2D, NAX)
        dc = dxn[:, G1D + G2D * NAX:] / m.sel
        # c_i = sum_j sw_ij g2b_ij g1_j[:32] / sel
        dg2b = dg2 + sw[:, None] * dc[src] * g1[dst, :G2D]
        np.add.at(dg1_in[:, :G2D], dst, sw[:, None] * dc[src] * g2b)
        dsw_acc += np.sum(dc[src] * g2b * g1[dst, :G2D], axis=1)
        # D = T T[:4]^T:  dT[m,a] = sum_b dD[m,b] T[b,a] + (m < 4) sum_m' dD[m',m] T[m',a]
        T = t["T"]
        dT = np.einsum("nmb,nba->nma", dD, T[:, :NAX, :])
        dT[:, :NAX, :] += np.einsum("nmb,nma->nba", dD, T)
        dT /= m.sel
        # T = sum_j g2b_j R_j^T / sel
        dg2b += np.einsum("ema,ea->em", dT[src], R)
        dR += np.einsum("ema,em->ea", dT[src], g2b)
        # attention, per centre
        dQ = np.zeros_like(t["Q"])
        dK = np.zeros_like(t["K"])
        dV = np.zeros_like(t["V"])
        for i in range(g["N"]):
            a, b = start[i], start[i + 1]
            rec = t["att"][i]
            if rec is None:
                continue
            dY = dg2b[a:b]
            dA = dY @ t["V"][a:b].T
            dV[a:b] = rec["A"].T @ dY
            dP = dA * rec["Gt"]
            dGt = dA * rec["P"]
            drh[a:b] += dGt @ rh[a:b] + dGt.T @ rh[a:b]
            rho = np.sum(dP * rec["P"], axis=1, keepdims=True)
            dsw_acc[a:b] += np.sum(rec["exZ"] * (dP - rho), axis=0)
            dS = rec["P"] * (dP - rho) / math.sqrt(G2D)
            dQ[a:b] = dS @ t["K"][a:b]
            dK[a:b] = dS.T @ t["Q"][a:b]
        dg2a = dg2b + dQ @ p[f"Wq{l}"].T + dK @ p[f"Wk{l}"].T + dV @ p[f"Wv{l}"].T
        # pair update: g2a = g2 + tanh([g2, g1_j] Wa + ba)
        dza = dg2a * (1.0 - t["ta"] ** 2)
        dxa = dza @ p[f"Wa{l}"].T
        dg2 = dg2a + dxa[:, :G2D]
        np.add.at(dg1_in, dst, dxa[:, G2D:])
        dg1 = dg1_in
    # g2 init = tanh(s Wp0 + bp0); R = (s, s rhat)
    g20 = f["tape"][0]["g2"]
    ds = np.sum(dg2 * (1.0 - g20 * g20) * p["Wp0"][0], axis=1) + dR[:, 0] + np.sum(dR[:, 1:] * rh, axis=1)
    drh += s[:, None] * dR[:, 1:]
    dr = ds * (dsw / r - sw / (r * r)) + dsw_acc * dsw
    proj = np.sum(drh * rh, axis=1)
    gD = dr[:, None] * rh + (drh - proj[:, None] * rh) / r[:, None]
    return Ei, gD


def evaluate(m: RepModel, X, types, box):
    """E, E_i, F [N][3] and the virial of the repformer model."""
    g = build_edges(m, X, types, box)
    Ei, gD = pair_gradients(m, g)
    F = np.zeros((g["N"], 3))
    np.add.at(F, g["src"], gD)
    np.subtract.at(F, g["dst"], gD)
    vir = -np.einsum("ea,eb->ab", g["D"], gD)
    return dict(E=math.fsum(Ei.tolist()), E_i=Ei, F=F, virial=vir, nlist=g["nlist"], nnei=g["nnei"])


def energy(m: RepModel, X, types, box):
    return math.fsum(forward(m, build_edges(m, X, types, box)).tolist())
