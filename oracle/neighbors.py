"""Neighbour lists within the model cutoff (oracle side).

The paper's models see each atom's neighbours within a cutoff (0.6 nm, i.e.
6 A; Section IV) through Verlet neighbour lists over periodic boundaries
(Section I-II).  The exact rule used here, so that two implementations can
agree bit for bit:

1. Delta_ij = x_j - x_i in float64;
2. periodic axis a: Delta_a <- Delta_a - L_a * rint(Delta_a * invL_a) with
   invL_a = 1/L_a computed once, rint rounding half to even, each product
   and difference rounded separately (no fused multiply-add);
3. d2 = (Dx*Dx + Dy*Dy) + Dz*Dz in that association;
4. j != i is a neighbour iff d2 < rc*rc (strict);
5. the list of i is sorted by ascending j;
6. if more than ``sel`` qualify, the ``sel`` smallest by (d2, j) are kept
   (then re-sorted by j) and the overflow is reported.

``neighbor_list_bruteforce`` is the plain O(N^2) definition;
``neighbor_list_cells`` reaches the same lists through a cell grid and is
checked against it.
"""
from __future__ import annotations

import math

import numpy as np


def _box_lengths(box):
    if box is None:
        return None
    box = np.asarray(box, dtype=np.float64)
    if box.shape == (3,):
        return box.copy()
    if np.any(box - np.diag(np.diag(box))):
        raise ValueError("only orthorhombic boxes are supported")
    return np.diag(box).copy()


def min_image(d: np.ndarray, L) -> np.ndarray:
    """Rule step 2 applied to an array of displacements [..., 3]."""
    if L is None:
        return d
    invL = 1.0 / L
    return d - L * np.rint(d * invL)


def dist2(d: np.ndarray) -> np.ndarray:
    """Rule step 3."""
    return (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]


def _finalise(js, d2, sel):
    """Rule steps 5-6 for one atom: js ascending candidate indices, d2 their squared distances."""
    if len(js) <= sel:
        return js, False
    order = np.lexsort((js, d2))[:sel]  # primary key d2, then j
    return np.sort(js[order]), True


def neighbor_list_bruteforce(X, box, rc: float, sel: int):
    """Plain O(N^2) search. Returns (nlist [N][sel] int32 padded with -1, nnei [N], n_overflow)."""
    X = np.asarray(X, dtype=np.float64)
    L = _box_lengths(box)
    N = X.shape[0]
    rc2 = rc * rc
    nlist = np.full((N, sel), -1, dtype=np.int32)
    nnei = np.zeros(N, dtype=np.int32)
    n_over = 0
    for i in range(N):
        d = min_image(X - X[i], L)
        d2 = dist2(d)
        mask = d2 < rc2
        mask[i] = False
        js = np.nonzero(mask)[0]
        js, over = _finalise(js, d2[js], sel)
        n_over += int(over)
        nlist[i, :len(js)] = js
        nnei[i] = len(js)
    return nlist, nnei, n_over


def neighbor_list_cells(X, box, rc: float, sel: int):
    """Cell-grid search with the same rule; must equal :func:`neighbor_list_bruteforce`."""
    X = np.asarray(X, dtype=np.float64)
    L = _box_lengths(box)
    N = X.shape[0]
    rc2 = rc * rc
    edge_min = rc * (1.0 + 1e-9)
    if L is not None:
        origin = np.zeros(3)
        ext = L
        W = X - L * np.floor(X / L)
    else:
        origin = X.min(0) if N else np.zeros(3)
        ext = (X.max(0) - origin) if N else np.ones(3)
        ext = np.maximum(ext, 1e-12)
        W = X - origin
    nc = np.maximum(1, np.floor(ext / edge_min).astype(int))
    cell = np.minimum(np.floor(W / (ext / nc)).astype(int), nc - 1)
    cell = np.maximum(cell, 0)
    buckets: dict[tuple, list] = {}
    for a in range(N):
        buckets.setdefault(tuple(cell[a]), []).append(a)
    nlist = np.full((N, sel), -1, dtype=np.int32)
    nnei = np.zeros(N, dtype=np.int32)
    n_over = 0
    for i in range(N):
        cells = set()
        for o in np.ndindex(3, 3, 3):
            c = cell[i] + np.array(o) - 1
            if L is not None:
                c = c % nc
            elif np.any(c < 0) or np.any(c >= nc):
                continue
            cells.add(tuple(int(v) for v in c))
        cand = sorted(j for c in cells for j in buckets.get(c, ()) if j != i)
        cand = np.array(cand, dtype=np.int64)
        if cand.size == 0:
            continue
        d = min_image(X[cand] - X[i], L)
        d2 = dist2(d)
        keep = d2 < rc2
        js, over = _finalise(cand[keep], d2[keep], sel)
        n_over += int(over)
        nlist[i, :len(js)] = js
        nnei[i] = len(js)
    return nlist, nnei, n_over


def cells_per_dim(box, rc: float):
    """Number of cells per axis a cell grid of edge >= rc gets (diagnostic)."""
    L = _box_lengths(box)
    return [max(1, int(math.floor(v / (rc * (1.0 + 1e-9))))) for v in L]
