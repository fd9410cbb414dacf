"""The GNN-variant descriptor in plain float64 NumPy, with a hand-written gradient --
TEST INFRASTRUCTURE ONLY (imported by tests and the smoke check, never by the library).

The paper's second model family (DPA3, Section II) replaces attention by graph
message passing over bonds and angles (a line-graph series).  It gives no
equations; this is the reading used here:

Graph.  Edges are the ordered pairs (i, j), j in N(i) (r_ij < rc = 6 A, the same
lists as the attention model).  Angles at centre i are the ordered pairs (j, k) of
distinct neighbours of i both within rca = 4 A.  Switches (quintic, smooth from
0.5 A): sw_e on [0.5, 6), sw_a on [0.5, 4).

Features.  node n_i (64), edge e_ij (64), angle a_ijk (32):
    n_i = TN[t_i];   s_ij = sw_e(r_ij) / r_ij;   e_ij = tanh(s_ij We0 + be0)
    c_ijk = rhat_ij . rhat_ik;   a_ijk = tanh(c_ijk Wa0 + ba0)
Three layers l = 0, 1, 2, each updating angles, then edges, then nodes:
    a_ijk <- a_ijk + tanh([a_ijk, e_ij[:32], e_ik[:32]] Waa_l + baa_l)
    m_ij   = sum_k sw_a(r_ij) sw_a(r_ik) tanh([a_ijk, e_ik[:32]] Wea_l + bea_l) / asel
    e_ij  <- e_ij + tanh([n_i, n_j, e_ij] Wee_l + bee_l) + m_ij
    n_i   <- n_i + tanh([n_i, sum_j sw_e(r_ij) e_ij / sel] Wnn_l + bnn_l)
(the angle update reads the layer's input edges, the edge update the updated angles
and the input nodes, the node update the updated edges).  Energy:
    y1 = tanh(n_i G1 + d1);  y2 = tanh(y1 G2 + d2) + y1;  E_i = y2 G3 + d3;  E = sum E_i
Every term an edge or angle adds is weighted by a switch that vanishes at its cutoff,
so E is smooth as atoms cross rc or rca.  E_i depends on atoms up to 3 rc away (each
layer's node update reads the neighbours' nodes of the layer before).

Gradient.  E depends on the positions only through the edge vectors Delta_ij (via
s_ij, sw_e, sw_a and rhat), so g_ij = dE/dDelta_ij (E the total energy) gives
F_i = sum_j g_ij - sum_j g_ji and the virial as for the attention model.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from .dp import switch
from .neighbors import neighbor_list_cells, min_image, _box_lengths

ND, ED, AD, NL = 64, 64, 32, 3  # node, edge, angle widths; layers
FH = 128  # fitting width


@dataclass
class GnnModel:
    ntypes: int = 5
    rc: float = 6.0
    rcs: float = 0.5
    rca: float = 4.0
    sel: int = 120
    asel: int = 48
    force_scale: float = 1.0
    p: dict = field(default_factory=dict)


def _shapes(ntypes, nd, ed, ad, nl, fh):
    out = [("TN", (ntypes, nd)), ("We0", (1, ed)), ("be0", (ed,)), ("Wa0", (1, ad)), ("ba0", (ad,))]
    for l in range(nl):
        out += [(f"Waa{l}", (ad + 64, ad)), (f"baa{l}", (ad,)), (f"Wea{l}", (ad + 32, ed)), (f"bea{l}", (ed,)),
                (f"Wee{l}", (2 * nd + ed, ed)), (f"bee{l}", (ed,)), (f"Wnn{l}", (nd + ed, nd)), (f"bnn{l}", (nd,))]
    out += [("G1", (nd, fh)), ("d1", (fh,)), ("G2", (fh, fh)), ("d2", (fh,)), ("G3", (fh, 1)), ("d3", (1,))]
    return out


def load_gnn_model(path: str) -> GnnModel:
    """Reads a GNN model file (magic DPGNNv01; the layout is described in synth/gnn_weights.py)."""
    import struct
    raw = open(path, "rb").read()
    if raw[:8] != b"DPGNNv01":
        raise ValueError("not a GNN model file")
    iv = struct.unpack_from("<16i", raw, 8)
    version, ntypes, nd, ed, ad, nl, fh, sel, asel = iv[:9]
    if version != 1 or (nd, ed, ad, nl, fh) != (ND, ED, AD, NL, FH):
        raise ValueError("unsupported GNN model file")
    rc, rcs, rca, fscale = struct.unpack_from("<4d", raw, 72)
    m = GnnModel(ntypes=ntypes, rc=rc, rcs=rcs, rca=rca, sel=sel, asel=asel, force_scale=fscale)
    off = 128
    for name, shape in _shapes(ntypes, nd, ed, ad, nl, fh):
        k = int(np.prod(shape))
        m.p[name] = np.frombuffer(raw, dtype="<f8", count=k, offset=off).reshape(shape).astype(np.float64)
        off += 8 * k
    if off != len(raw):
        raise ValueError("GNN model file size mismatch")
    return m


# ----------------------------------------------------------------------------- graph
def build_graph(m: GnnModel, X, types, box, nlist=None, nnei=None):
    """Edges (centre, neighbour, Delta) from the neighbour lists, and the angles of every
    centre as pairs of its edge indices (ep: edge i-j, eq: edge i-k), in list order."""
    X = np.asarray(X, dtype=np.float64)
    L = _box_lengths(box)
    if nlist is None:
        nlist, nnei, _ = neighbor_list_cells(X, box, m.rc, m.sel)
    src, dst = [], []
    for i in range(X.shape[0]):
        for j in nlist[i, :nnei[i]]:
            src.append(i)
            dst.append(int(j))
    src, dst = np.array(src, dtype=np.int64), np.array(dst, dtype=np.int64)
    D = min_image(X[dst] - X[src], L)
    r = np.sqrt(np.sum(D * D, axis=1))
    ep, eq = [], []
    start = np.concatenate([[0], np.cumsum(nnei)])
    for i in range(X.shape[0]):
        close = [e for e in range(start[i], start[i + 1]) if r[e] < m.rca][:m.asel]
        for p in close:
            for q in close:
                if p != q:
                    ep.append(p)
                    eq.append(q)
    return dict(src=src, dst=dst, D=D, ep=np.array(ep, dtype=np.int64), eq=np.array(eq, dtype=np.int64),
                types=np.asarray(types), N=X.shape[0], nlist=nlist, nnei=nnei)


def _edge_terms(m, D):
    r = np.sqrt(np.sum(D * D, axis=1))
    swe, dswe = switch(r, m.rc, m.rcs)
    swa, dswa = switch(r, m.rca, m.rcs)
    return r, swe, dswe, swa, dswa, D / r[:, None]


# ----------------------------------------------------------------------------- forward
def forward(m: GnnModel, g: dict, keep: bool = False):
    """Atomic energies E_i; with keep, also the intermediates the gradient needs."""
    p = m.p
    src, dst, ep, eq = g["src"], g["dst"], g["ep"], g["eq"]
    r, swe, _, swa, _, rh = _edge_terms(m, g["D"])
    s = swe / r
    n = p["TN"][g["types"]]
    e = np.tanh(s[:, None] * p["We0"][0] + p["be0"])
    c = np.sum(rh[ep] * rh[eq], axis=1)
    a = np.tanh(c[:, None] * p["Wa0"][0] + p["ba0"])
    wa = swa[ep] * swa[eq] / m.asel
    tape = []
    for l in range(NL):
        xa = np.concatenate([a, e[ep, :32], e[eq, :32]], axis=1)
        ta = np.tanh(xa @ p[f"Waa{l}"] + p[f"baa{l}"])
        a1 = a + ta
        xm = np.concatenate([a1, e[eq, :32]], axis=1)
        tm = np.tanh(xm @ p[f"Wea{l}"] + p[f"bea{l}"])
        msg = tm * wa[:, None]
        mm = np.zeros_like(e)
        np.add.at(mm, ep, msg)
        xe = np.concatenate([n[src], n[dst], e], axis=1)
        te = np.tanh(xe @ p[f"Wee{l}"] + p[f"bee{l}"])
        e1 = e + te + mm
        agg = np.zeros_like(n)
        np.add.at(agg, src, swe[:, None] * e1)
        agg /= m.sel
        xn = np.concatenate([n, agg], axis=1)
        tn = np.tanh(xn @ p[f"Wnn{l}"] + p[f"bnn{l}"])
        n1 = n + tn
        tape.append(dict(a=a, e=e, n=n, xa=xa, ta=ta, a1=a1, xm=xm, tm=tm, xe=xe, te=te, e1=e1, agg=agg, xn=xn,
                         tn=tn))
        a, e, n = a1, e1, n1
    y1 = np.tanh(n @ p["G1"] + p["d1"])
    y2 = np.tanh(y1 @ p["G2"] + p["d2"]) + y1
    Ei = (y2 @ p["G3"])[:, 0] + p["d3"][0]
    if not keep:
        return Ei
    return Ei, dict(tape=tape, n=n, y1=y1, y2=y2, r=r, s=s, swe=swe, swa=swa, rh=rh, c=c, wa=wa)


# ----------------------------------------------------------------------------- gradient
def pair_gradients(m: GnnModel, g: dict):
    """E_i and g_e = dE/dDelta_e for every edge e (E the total energy), reverse mode."""
    p = m.p
    src, dst, ep, eq = g["src"], g["dst"], g["ep"], g["eq"]
    Ei, f = forward(m, g, keep=True)
    r, s, swe, swa, rh, c, wa = f["r"], f["s"], f["swe"], f["swa"], f["rh"], f["c"], f["wa"]
    _, _, dswe, _, dswa, _ = _edge_terms(m, g["D"])
    # fitting: dE/dn with dE/dE_i = 1
    dy2 = np.broadcast_to(p["G3"][:, 0], f["y2"].shape).copy()
    t2 = f["y2"] - f["y1"]
    dp2 = dy2 * (1.0 - t2 * t2)
    dy1 = dp2 @ p["G2"].T + dy2
    dp1 = dy1 * (1.0 - f["y1"] ** 2)
    dn = dp1 @ p["G1"].T
    de = np.zeros((len(src), ED))
    da = np.zeros((len(ep), AD))
    dswe_acc = np.zeros(len(src))   # dE/dsw_e per edge
    dwa = np.zeros(len(ep))         # dE/dwa per angle
    for l in reversed(range(NL)):
        t = f["tape"][l]
        # node update: n1 = n + tanh(xn Wnn + b)
        dpn = dn * (1.0 - t["tn"] ** 2)
        dxn = dpn @ p[f"Wnn{l}"].T
        dn_in = dn + dxn[:, :ND]
        dagg = dxn[:, ND:] / m.sel
        # agg_i = sum_e swe_e e1_e over edges of i
        de1 = de + swe[:, None] * dagg[src]
        dswe_acc += np.sum(t["e1"] * dagg[src], axis=1)
        # edge update: e1 = e + te + mm
        dpe = de1 * (1.0 - t["te"] ** 2)
        dxe = dpe @ p[f"Wee{l}"].T
        de_in = de1 + dxe[:, 2 * ND:]
        np.add.at(dn_in, src, dxe[:, :ND])
        np.add.at(dn_in, dst, dxe[:, ND:2 * ND])
        # mm_e = sum over angles with ep = e of msg
        dmsg = de1[ep]
        dwa += np.sum(dmsg * t["tm"], axis=1)
        dtm = dmsg * wa[:, None]
        dpm = dtm * (1.0 - t["tm"] ** 2)
        dxm = dpm @ p[f"Wea{l}"].T
        da1 = da + dxm[:, :AD]
        np.add.at(de_in[:, :32], eq, dxm[:, AD:])
        # angle update: a1 = a + tanh(xa Waa + b)
        dpa = da1 * (1.0 - t["ta"] ** 2)
        dxa = dpa @ p[f"Waa{l}"].T
        da = da1 + dxa[:, :AD]
        np.add.at(de_in[:, :32], ep, dxa[:, AD:AD + 32])
        np.add.at(de_in[:, :32], eq, dxa[:, AD + 32:])
        de, dn = de_in, dn_in
    # initial features: e = tanh(s We0 + be0), a = tanh(c Wa0 + ba0)
    e0 = f["tape"][0]["e"]
    a0 = f["tape"][0]["a"]
    ds = np.sum(de * (1.0 - e0 * e0) * p["We0"][0], axis=1)
    dc = np.sum(da * (1.0 - a0 * a0) * p["Wa0"][0], axis=1)
    # wa = swa[ep] swa[eq] / asel
    dswa_acc = np.zeros(len(src))
    np.add.at(dswa_acc, ep, dwa * swa[eq] / m.asel)
    np.add.at(dswa_acc, eq, dwa * swa[ep] / m.asel)
    # c = rh[ep] . rh[eq]
    drh = np.zeros_like(rh)
    np.add.at(drh, ep, dc[:, None] * rh[eq])
    np.add.at(drh, eq, dc[:, None] * rh[ep])
    # edge scalars -> Delta:  s = swe / r;  rh = D / r
    dr = ds * (dswe / r - swe / (r * r)) + dswe_acc * dswe + dswa_acc * dswa
    proj = np.sum(drh * rh, axis=1)
    gD = dr[:, None] * rh + (drh - proj[:, None] * rh) / r[:, None]
    return Ei, gD


def evaluate(m: GnnModel, X, types, box):
    """E, E_i, F [N][3] and the virial of the GNN model."""
    g = build_graph(m, X, types, box)
    Ei, gD = pair_gradients(m, g)
    F = np.zeros((g["N"], 3))
    np.add.at(F, g["src"], gD)
    np.subtract.at(F, g["dst"], gD)
    vir = -np.einsum("ea,eb->ab", g["D"], gD)
    return dict(E=math.fsum(Ei.tolist()), E_i=Ei, F=F, virial=vir, nlist=g["nlist"], nnei=g["nnei"],
                n_angles=len(g["ep"]))


def energy(m: GnnModel, X, types, box):
    return math.fsum(forward(m, build_graph(m, X, types, box)).tolist())
