"""The deep-potential model in plain float64 NumPy, with a hand-written gradient.

Reading of the paper (Section II names the parts; the sizes are those of the
attention model studied here; the functional form is the reading recorded in
the model definition below):

Environment, per neighbour j of atom i (Delta = x_j - x_i, r = |Delta|):
    u = (r - rcs) / (rc - rcs);  sw = 1 for r < rcs, u^3 (-6u^2 + 15u - 10) + 1 below rc
    s = sw / r;  rhat = Delta / r;  Rt_j = (s, s rhat_x, s rhat_y, s rhat_z)
Type-embedded embedding net (17 -> 25 -> 50 -> 100, tanh, residual [h, h]):
    z = [s, TE[t_j], TE[t_i]];  h1 = tanh(z W1 + b1)
    h2 = tanh(h1 W2 + b2) + [h1, h1];  G_j = tanh(h2 W3 + b3) + [h2, h2]
Gated self-attention over the neighbours of i (tokens = neighbours), twice:
    Q, K, V = G WQ, G WK, G WV;  S = Q K^T / sqrt(d);  m_j = max_k S_jk
    P_jk = sw_k exp(S_jk - m_j) / sum_k' sw_k' exp(S_jk' - m_j)
    A_jk = P_jk (rhat_j . rhat_k);  Y = (A V) WO
    X = G + Y;  G <- gamma * (X - mean(X)) / sqrt(var(X) + eps) + beta   (population variance, per token)
Descriptor:  T = G^T Rt / sel  [M x 4];  D = T T_{<M2}^T  [M x M2], flattened row-major (16 m + a)
Fitting (1600 -> 240 -> 240 -> 240 -> 1):
    y1 = tanh(D F1 + c1);  y2 = tanh(y1 F2 + c2) + y1;  y3 = tanh(y2 F3 + c3) + y2
    E_i = y3 F4 + c4 + ebias[t_i];   E = sum_i E_i (correctly rounded, math.fsum)
Gradient g_ij = dE_i/dDelta_ij by reverse mode; forces
    F_i = sum_{j in N(i)} g_ij - sum_{j : i in N(j)} g_ji   (F = -dE/dx)
and virial  Xi_ab = - sum_i sum_{j in N(i)} Delta_ij,a g_ij,b.
"""
from __future__ import annotations

import math

import numpy as np

from .neighbors import neighbor_list_bruteforce, neighbor_list_cells, min_image, _box_lengths


# ----------------------------------------------------------------------------- switch
def switch(r, rc: float, rcs: float):
    """Quintic smooth switch sw(r) and its derivative dsw/dr (C2 at rcs and rc)."""
    r = np.asarray(r, dtype=np.float64)
    u = (r - rcs) / (rc - rcs)
    inside = (r >= rcs) & (r < rc)
    sw = np.where(r < rcs, 1.0, np.where(inside, u ** 3 * (-6.0 * u ** 2 + 15.0 * u - 10.0) + 1.0, 0.0))
    dsw = np.where(inside, -30.0 * u ** 2 * (1.0 - u) ** 2 / (rc - rcs), 0.0)
    return sw, dsw


# ----------------------------------------------------------------------------- one atom
def atom_energy_and_grad(m, t_i: int, t_j: np.ndarray, dR: np.ndarray, want_grad: bool = True,
                         keep: dict | None = None):
    """Energy E_i of one atom and g = dE_i/dDelta_ij for its n neighbours (dR [n][3]).

    ``keep``, when a dict, receives the intermediates (env, G after each stage, T, D).
    """
    p = m.p
    n = dR.shape[0]
    M, M2, d = m.M, m.M2, m.d_attn
    dR = np.asarray(dR, dtype=np.float64)
    # -- environment
    r = np.sqrt(np.sum(dR * dR, axis=1))
    sw, dsw = switch(r, m.rc, m.rcs)
    s = sw / r
    rhat = dR / r[:, None]
    Rt = np.concatenate([s[:, None], s[:, None] * rhat], axis=1)
    # -- embedding net
    z = np.concatenate([s[:, None], p["TE"][t_j], np.broadcast_to(p["TE"][t_i], (n, m.tebd))], axis=1)
    h1 = np.tanh(z @ p["W1"] + p["b1"])
    t2 = np.tanh(h1 @ p["W2"] + p["b2"])
    h2 = t2 + np.concatenate([h1, h1], axis=1)
    t3 = np.tanh(h2 @ p["W3"] + p["b3"])
    G = t3 + np.concatenate([h2, h2], axis=1)
    if keep is not None:
        keep.update(r=r, sw=sw, s=s, rhat=rhat, Rt=Rt, G0=G.copy())
    # -- attention layers
    C = rhat @ rhat.T  # gate: rhat_j . rhat_k
    saved = []
    for a in range(m.n_attn):
        Gin = G
        Q = Gin @ p[f"WQ{a}"]
        K = Gin @ p[f"WK{a}"]
        V = Gin @ p[f"WV{a}"]
        S = (Q @ K.T) / math.sqrt(d)
        mrow = S.max(axis=1, keepdims=True) if n else S
        Ex = np.exp(S - mrow)              # exp(S_jk - m_j)
        e = Ex * sw[None, :]               # sw_k exp(S_jk - m_j)
        Z = e.sum(axis=1, keepdims=True)
        P = e / Z
        A = P * C
        O = A @ V
        Y = O @ p[f"WO{a}"]
        X = Gin + Y                        # residual, then LayerNorm over the features
        mu = X.mean(axis=1, keepdims=True)
        var = ((X - mu) ** 2).mean(axis=1, keepdims=True)
        sig = np.sqrt(var + m.ln_eps)
        Xh = (X - mu) / sig
        G = p[f"gamma{a}"] * Xh + p[f"beta{a}"]
        saved.append((Gin, Q, K, V, Ex, Z, P, A, sig, Xh))
        if keep is not None:
            keep[f"G{a + 1}"] = G.copy()
    # -- descriptor
    T = G.T @ Rt / m.sel               # [M][4]
    D = T @ T[:M2].T                   # [M][M2]
    x = D.reshape(-1)
    # -- fitting net
    y1 = np.tanh(x @ p["F1"] + p["c1"])
    t2f = np.tanh(y1 @ p["F2"] + p["c2"])
    y2 = t2f + y1
    t3f = np.tanh(y2 @ p["F3"] + p["c3"])
    y3 = t3f + y2
    Ei = float((y3 @ p["F4"])[0] + p["c4"][0] + p["ebias"][t_i])
    if keep is not None:
        keep.update(T=T, D=D, y1=y1, y2=y2, y3=y3)
    if not want_grad:
        return Ei, None
    # ======================================================== reverse mode, dE_i = 1
    dy3 = p["F4"][:, 0].copy()
    dpre = dy3 * (1.0 - t3f ** 2)
    dy2 = dpre @ p["F3"].T + dy3
    dpre = dy2 * (1.0 - t2f ** 2)
    dy1 = dpre @ p["F2"].T + dy2
    dpre = dy1 * (1.0 - y1 ** 2)
    dx = dpre @ p["F1"].T
    dD = dx.reshape(M, M2)
    # D = T T_<M2^T:  dT_m += sum_a dD_ma T_a ;  dT_a += sum_m dD_ma T_m  (a < M2)
    dT = dD @ T[:M2]
    dT[:M2] += dD.T @ T
    dG = Rt @ dT.T / m.sel             # [n][M]
    dRt = G @ dT / m.sel               # [n][4]
    drhat = np.zeros_like(rhat)
    dsw_acc = np.zeros(n)
    for a in reversed(range(m.n_attn)):
        Gin, Q, K, V, Ex, Z, P, A, sig, Xh = saved[a]
        dXh = dG * p[f"gamma{a}"]
        dX = (dXh - dXh.mean(axis=1, keepdims=True)
              - Xh * (dXh * Xh).mean(axis=1, keepdims=True)) / sig
        dGin = dX.copy()                                   # residual path (through the LayerNorm)
        dY = dX
        dO = dY @ p[f"WO{a}"].T
        dA = dO @ V.T
        dV = A.T @ dO
        dP = dA * C
        dC = dA * P
        drhat += dC @ rhat + dC.T @ rhat
        rho = (P * dP).sum(axis=1, keepdims=True)
        Wt = (Ex / Z) * (dP - rho)                         # never divides by sw
        dS = Wt * sw[None, :]
        dsw_acc += Wt.sum(axis=0)
        dS /= math.sqrt(d)
        dQ = dS @ K
        dK = dS.T @ Q
        dGin += dQ @ p[f"WQ{a}"].T + dK @ p[f"WK{a}"].T + dV @ p[f"WV{a}"].T
        dG = dGin
    # embedding backward
    dpre3 = dG * (1.0 - t3 ** 2)
    dh2 = dpre3 @ p["W3"].T + dG[:, :m.e2] + dG[:, m.e2:]
    dpre2 = dh2 * (1.0 - t2 ** 2)
    dh1 = dpre2 @ p["W2"].T + dh2[:, :m.e1] + dh2[:, m.e1:]
    dpre1 = dh1 * (1.0 - h1 ** 2)
    ds = dpre1 @ p["W1"][0]
    # Rt = (s, s rhat)
    ds += dRt[:, 0] + np.sum(dRt[:, 1:] * rhat, axis=1)
    drhat += s[:, None] * dRt[:, 1:]
    # s = sw / r
    dsw_acc += ds / r
    dr = -ds * sw / r ** 2 + dsw_acc * dsw
    # rhat = Delta / r,  r = |Delta|
    g = (drhat - np.sum(drhat * rhat, axis=1, keepdims=True) * rhat) / r[:, None] + dr[:, None] * rhat
    return Ei, g


# ----------------------------------------------------------------------------- systems
def _pair_vectors(X, L, i, js):
    return min_image(X[js] - X[i], L)


def evaluate_subset(m, X, types, box, centers, nlist=None, nnei=None):
    """E_i, neighbour indices and g_ij for the given centre atoms only.

    Returns (E_i [k], list of neighbour index arrays, list of g arrays [n_i][3],
    list of Delta arrays [n_i][3]).
    """
    X = np.asarray(X, dtype=np.float64)
    L = _box_lengths(box)
    if nlist is None:
        nlist, nnei, _ = neighbor_list_cells(X, box, m.rc, m.sel)
    Es, nbrs, gs, ds = [], [], [], []
    for i in centers:
        js = nlist[i, :nnei[i]].astype(np.int64)
        dR = _pair_vectors(X, L, i, js)
        Ei, g = atom_energy_and_grad(m, int(types[i]), types[js], dR)
        Es.append(Ei)
        nbrs.append(js)
        gs.append(g)
        ds.append(dR)
    return np.array(Es), nbrs, gs, ds


def forces_from_pairs(N, nbrs, gs, centers=None):
    """F_i = sum_j g_ij - sum_{j: i in N(j)} g_ji by gather over every evaluated centre."""
    F = np.zeros((N, 3))
    centers = range(N) if centers is None else centers
    for i, js, g in zip(centers, nbrs, gs):
        F[i] += g.sum(axis=0)
        np.subtract.at(F, js, g)
    return F


def evaluate(m, X, types, box, neighbor_search: str = "cells"):
    """Full evaluation: dict with E, E_i, F [N][3], virial [3][3], nlist, nnei, n_overflow."""
    X = np.asarray(X, dtype=np.float64)
    N = X.shape[0]
    search = neighbor_list_cells if neighbor_search == "cells" else neighbor_list_bruteforce
    nlist, nnei, n_over = search(X, box, m.rc, m.sel)
    Ei, nbrs, gs, ds = evaluate_subset(m, X, types, box, range(N), nlist, nnei)
    F = forces_from_pairs(N, nbrs, gs)
    allD = np.concatenate(ds, 0) if ds else np.zeros((0, 3))
    allg = np.concatenate(gs, 0) if gs else np.zeros((0, 3))
    vir = np.zeros((3, 3))
    for a in range(3):
        for b in range(3):
            vir[a, b] = -math.fsum((allD[:, a] * allg[:, b]).tolist())
    return dict(E=math.fsum(Ei.tolist()), E_i=Ei, F=F, virial=vir, nlist=nlist, nnei=nnei,
                n_overflow=n_over)


def energy_only(m, X, types, box):
    """Total energy without gradients (for finite differences)."""
    X = np.asarray(X, dtype=np.float64)
    L = _box_lengths(box)
    nlist, nnei, _ = neighbor_list_cells(X, box, m.rc, m.sel)
    out = []
    for i in range(X.shape[0]):
        js = nlist[i, :nnei[i]].astype(np.int64)
        Ei, _ = atom_energy_and_grad(m, int(types[i]), types[js], _pair_vectors(X, L, i, js), want_grad=False)
        out.append(Ei)
    return math.fsum(out)


def local_energy(m, X, types, box, atoms):
    """Sum of E_i over the given atoms (finite differences that touch one atom only need its neighbourhood)."""
    X = np.asarray(X, dtype=np.float64)
    L = _box_lengths(box)
    nlist, nnei, _ = neighbor_list_cells(X, box, m.rc, m.sel)
    out = []
    for i in atoms:
        js = nlist[i, :nnei[i]].astype(np.int64)
        Ei, _ = atom_energy_and_grad(m, int(types[i]), types[js], _pair_vectors(X, L, i, js), want_grad=False)
        out.append(Ei)
    return math.fsum(out)


# ----------------------------------------------------------------------------- fitting heads
def head_view(m, h: int):
    """The model with fitting head h in place of head 0; every other array is shared.

    Several fitting nets on one descriptor (the paper's multi-task models, Section II,
    share one descriptor between branches): head h maps the same D to its own E_i^h.
    """
    import copy
    v = copy.copy(m)
    v.p = dict(m.p)
    v.p.update(m.heads[h])
    return v


def evaluate_heads(m, X, types, box, weights):
    """Energy, forces and virial of the weighted head combination E = sum_h w_h E^h, plus
    every head's total energy.  Each head is a plain evaluation of its own model view;
    forces and virial are linear in the energy, so they combine with the same weights."""
    out = {"E_heads": [], "E": 0.0, "F": 0.0, "virial": 0.0, "E_i": 0.0}
    for h in range(len(m.heads)):
        r = evaluate(head_view(m, h), X, types, box)
        out["E_heads"].append(r["E"])
        w = float(weights[h])
        out["E"] = out["E"] + w * r["E"]
        out["F"] = out["F"] + w * r["F"]
        out["virial"] = out["virial"] + w * r["virial"]
        out["E_i"] = out["E_i"] + w * r["E_i"]
    out["E_heads"] = np.array(out["E_heads"])
    return out
