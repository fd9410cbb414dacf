"""A second, scalar-loop evaluation of one atom's energy, for tiny neighbourhoods.

Every quantity is computed element by element with Python floats or mpmath
numbers (``num`` selects the number type), with no matrix library, so that a
transposed operand, a wrong index or a dropped term in the vectorised oracle
shows up as a mismatch.  It follows the same reading of the model: quintic
switch, environment row (s, s rhat), [s, TE[t_j], TE[t_i]] embedding with
[h, h] residuals, switch-weighted gated softmax attention with a residual update
followed by LayerNorm, 1/sel descriptor T and D = T T_<M2^T, fitting net with
residuals on the hidden layers.
"""
import math


def atom_energy_scalar(m, t_i, t_j, dR, num=float, tanh=math.tanh, exp=math.exp, sqrt=math.sqrt):
    p = m.p
    n = len(dR)
    M, M2, d = m.M, m.M2, m.d_attn
    rc, rcs = num(m.rc), num(m.rcs)

    def N(x):
        return num(float(x)) if num is not float else float(x)

    r, s, sw, rh = [], [], [], []
    for j in range(n):
        x, y, z = (num(dR[j][0]), num(dR[j][1]), num(dR[j][2]))
        rr = sqrt(x * x + y * y + z * z)
        if rr < rcs:
            w = num(1)
        elif rr < rc:
            u = (rr - rcs) / (rc - rcs)
            w = u ** 3 * (-6 * u ** 2 + 15 * u - 10) + 1
        else:
            w = num(0)
        r.append(rr)
        sw.append(w)
        s.append(w / rr)
        rh.append((x / rr, y / rr, z / rr))
    Rt = [[s[j], s[j] * rh[j][0], s[j] * rh[j][1], s[j] * rh[j][2]] for j in range(n)]

    def dense(vec, W, b, nin, nout):
        out = []
        for o in range(nout):
            acc = N(b[o]) if b is not None else num(0)
            for i in range(nin):
                acc += vec[i] * N(W[i][o])
            out.append(acc)
        return out

    G = []
    for j in range(n):
        z = [s[j]] + [N(v) for v in p["TE"][t_j[j]]] + [N(v) for v in p["TE"][t_i]]
        h1 = [tanh(v) for v in dense(z, p["W1"], p["b1"], 1 + 2 * m.tebd, m.e1)]
        a2 = dense(h1, p["W2"], p["b2"], m.e1, m.e2)
        h2 = [tanh(a2[o]) + h1[o % m.e1] for o in range(m.e2)]
        a3 = dense(h2, p["W3"], p["b3"], m.e2, M)
        G.append([tanh(a3[o]) + h2[o % m.e2] for o in range(M)])

    for a in range(m.n_attn):
        Q = [dense(G[j], p[f"WQ{a}"], None, M, d) for j in range(n)]
        K = [dense(G[j], p[f"WK{a}"], None, M, d) for j in range(n)]
        V = [dense(G[j], p[f"WV{a}"], None, M, d) for j in range(n)]
        newG = []
        for j in range(n):
            Srow = []
            for k in range(n):
                acc = num(0)
                for c in range(d):
                    acc += Q[j][c] * K[k][c]
                Srow.append(acc / sqrt(num(d)))
            mx = max(Srow)
            e = [sw[k] * exp(Srow[k] - mx) for k in range(n)]
            Z = sum(e)
            O = [num(0)] * d
            for k in range(n):
                gate = rh[j][0] * rh[k][0] + rh[j][1] * rh[k][1] + rh[j][2] * rh[k][2]
                w = e[k] / Z * gate
                for c in range(d):
                    O[c] += w * V[k][c]
            Y = dense(O, p[f"WO{a}"], None, d, M)
            X = [G[j][o] + Y[o] for o in range(M)]
            mu = sum(X) / M
            var = sum((x - mu) ** 2 for x in X) / M
            sg = sqrt(var + num(m.ln_eps))
            newG.append([N(p[f"gamma{a}"][o]) * (X[o] - mu) / sg + N(p[f"beta{a}"][o]) for o in range(M)])
        G = newG

    T = [[sum(G[j][mm] * Rt[j][c] for j in range(n)) / m.sel for c in range(4)] for mm in range(M)]
    x = []
    for mm in range(M):
        for aa in range(M2):
            x.append(sum(T[mm][c] * T[aa][c] for c in range(4)))
    H = m.fit_hidden
    y = [tanh(v) for v in dense(x, p["F1"], p["c1"], M * M2, H)]
    for li in (2, 3):
        a_ = dense(y, p[f"F{li}"], p[f"c{li}"], H, H)
        y = [tanh(a_[o]) + y[o] for o in range(H)]
    E = N(p["c4"][0]) + N(p["ebias"][t_i])
    for o in range(H):
        E += y[o] * N(p["F4"][o][0])
    return E
