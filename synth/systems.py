"""Seeded protein-in-water-shaped systems.

The paper measures four solvated proteins (Section IV).  Their structures are
not available here, so seeded synthetic stand-ins take their place: periodic
cubic boxes of rigid-geometry water at 1 g/cm^3, optionally with a
self-avoiding solute chain whose atom types follow a protein-like ratio
C:N:O:H:S = 32:9:10:48:1.  Every atom is a deep-potential atom.

Recipe (all lengths in Angstrom, masses in amu):

* water: O at the origin, two H at 0.96 A, H-O-H angle 104.5 deg, a uniformly
  random orientation (unit quaternion from four normal draws);
* water O positions by random sequential insertion with a periodic
  O-O distance >= 2.5 A (grid-accelerated);
* chain: self-avoiding walk from the box centre, bond length ~ U(1.0, 1.5),
  direction uniform on the sphere; a step is rejected if it lands within
  1.6 A of any earlier non-bonded chain atom (periodic), up to 200 retries,
  after which the walk backs off one atom;
* solvation: L is chosen so that (chain mass + W * 18.015) / L^3 equals
  0.602214 amu/A^3 (1 g/cm^3) with W = round((N_target - N_chain) / 3);
  waters whose atoms come within 2.0 A of a chain atom are rejected.

Type indices: O=0, H=1, C=2, N=3, S=4.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

TYPE_NAMES = ("O", "H", "C", "N", "S")
TYPE_INDEX = {n: i for i, n in enumerate(TYPE_NAMES)}
MASSES = np.array([15.999, 1.008, 12.011, 14.007, 32.06])  # amu, by type index
WATER_MASS = 18.015
DENSITY_AMU_PER_A3 = 0.602214  # 1 g/cm^3

OH_BOND = 0.96
HOH_ANGLE = math.radians(104.5)
OO_MIN = 2.5
CHAIN_WATER_MIN = 2.0
CHAIN_NONBONDED_MIN = 1.6
CHAIN_RATIO = (("C", 32), ("N", 9), ("O", 10), ("H", 48), ("S", 1))


@dataclass
class System:
    """Positions [N][3] (float64, A), types [N] (int32), cubic box edge L (A)."""

    coords: np.ndarray
    types: np.ndarray
    box: np.ndarray  # [3][3] row vectors (diagonal)
    n_chain: int = 0
    n_water: int = 0

    @property
    def natoms(self) -> int:
        return int(self.coords.shape[0])


def _random_rotations(rng: np.random.Generator, k: int) -> np.ndarray:
    q = rng.normal(size=(k, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)], -1),
        np.stack([2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)], -1),
        np.stack([2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)], -1),
    ], 1)


def _water_template() -> np.ndarray:
    half = HOH_ANGLE / 2
    return np.array([
        [0.0, 0.0, 0.0],
        [OH_BOND * math.sin(half), OH_BOND * math.cos(half), 0.0],
        [-OH_BOND * math.sin(half), OH_BOND * math.cos(half), 0.0],
    ])


class _Grid:
    """Periodic bucket grid used to reject insertions that come too close.

    The points are kept twice: in per-cell lists (the exact scalar test) and in a
    NaN-padded array [n][n][n][K][3] for a vectorised test of many candidates at once.
    """

    def __init__(self, L: float, cell: float, k_max: int = 8):
        self.L = L
        self.n = max(1, int(L // cell))
        self.cell = L / self.n
        self.buckets: dict[tuple, list] = {}
        self.arr = np.full((self.n, self.n, self.n, k_max, 3), np.nan)
        self.cnt = np.zeros((self.n, self.n, self.n), dtype=np.int64)

    def _key(self, p):
        c = np.floor((p % self.L) / self.cell).astype(int) % self.n
        return int(c[0]), int(c[1]), int(c[2])

    def add(self, p):
        p = np.asarray(p, dtype=float)
        key = self._key(p)
        self.buckets.setdefault(key, []).append(p)
        k = self.cnt[key]
        if k >= self.arr.shape[3]:  # grow the padded array
            grown = np.full(self.arr.shape[:3] + (2 * self.arr.shape[3], 3), np.nan)
            grown[:, :, :, :self.arr.shape[3]] = self.arr
            self.arr = grown
        self.arr[key][k] = p
        self.cnt[key] += 1

    def too_close(self, p, dmin: float) -> bool:
        cx, cy, cz = self._key(p)
        reach = int(math.ceil(dmin / self.cell))
        n = self.n
        seen = set()
        for ox in range(-reach, reach + 1):
            for oy in range(-reach, reach + 1):
                for oz in range(-reach, reach + 1):
                    key = ((cx + ox) % n, (cy + oy) % n, (cz + oz) % n)
                    if key in seen:
                        continue
                    seen.add(key)
                    for q in self.buckets.get(key, ()):
                        d = q - p
                        d -= self.L * np.rint(d / self.L)
                        if d @ d < dmin * dmin:
                            return True
        return False

    def too_close_many(self, P, dmin: float) -> np.ndarray:
        """too_close for each row of P, against the points present now.  The vectorised
        squared distances decide every clear case; a candidate within a relative 1e-9 of
        the limit is decided by the scalar test, so the answers are exactly too_close's."""
        P = np.asarray(P, dtype=float)
        reach = int(math.ceil(dmin / self.cell))
        n = self.n
        c = np.floor((P % self.L) / self.cell).astype(int) % n
        if getattr(self, "_stencil", (None,))[0] != reach:
            offs = np.arange(-reach, reach + 1)
            ox, oy, oz = np.meshgrid(offs, offs, offs, indexing="ij")
            self._stencil = (reach, np.stack([ox.ravel(), oy.ravel(), oz.ravel()], 1))
        cells = (c[:, None, :] + self._stencil[1][None]) % n                                   # [m][27][3]
        # a cell reached twice (n < 2 reach + 1) holds the same points: counting them twice is harmless
        kmax = max(1, int(self.cnt.max()))
        Q = self.arr[cells[..., 0], cells[..., 1], cells[..., 2], :kmax]                        # [m][27][K][3]
        d = Q - P[:, None, None, :]
        d -= self.L * np.rint(d / self.L)
        d2 = np.sum(d * d, axis=-1)
        lim = dmin * dmin
        with np.errstate(invalid="ignore"):
            close = np.any(d2 < lim * (1.0 - 1e-9), axis=(1, 2))
            edge = np.any(np.abs(d2 - lim) <= lim * 1e-9, axis=(1, 2)) & ~close
        for i in np.nonzero(edge)[0]:
            close[i] = self.too_close(P[i], dmin)
        return close


def _insert_waters(rng, L, n_water, chain_grid=None, max_tries=2000):
    """Random sequential insertion of rigid waters.  Each batch of candidates is first
    tested against the oxygens already placed (vectorised); the survivors are then taken
    in order, each tested against the oxygens accepted earlier in the same batch and
    against the chain, exactly as a one-by-one insertion would."""
    tmpl = _water_template()
    o_grid = _Grid(L, OO_MIN)
    out = []
    batch = 256
    lim = OO_MIN * OO_MIN
    while len(out) < n_water:
        cand = rng.uniform(0.0, L, size=(batch, 3))
        rots = _random_rotations(rng, batch)
        free = np.nonzero(~o_grid.too_close_many(cand, OO_MIN))[0]
        # clash[a, b]: free candidates a and b closer than OO_MIN (decided as too_close does)
        F = cand[free]
        d = F[:, None, :] - F[None, :, :]
        d -= L * np.rint(d / L)
        d2 = np.sum(d * d, axis=-1)
        clash = d2 < lim * (1.0 - 1e-9)
        for a, b in zip(*np.nonzero((np.abs(d2 - lim) <= lim * 1e-9) & ~clash)):
            e = F[a] - F[b]
            e -= L * np.rint(e / L)
            clash[a, b] = e @ e < lim
        mols = [cand[k] + tmpl @ rots[k].T for k in free]
        if chain_grid is not None and len(free):
            wet = chain_grid.too_close_many(np.concatenate(mols, 0), CHAIN_WATER_MIN).reshape(-1, 3).any(1)
        else:
            wet = np.zeros(len(free), dtype=bool)
        taken = []
        for a, k in enumerate(free):
            if len(out) >= n_water:
                break
            if taken and clash[taken, a].any():
                continue
            mol = mols[a]
            if wet[a]:
                continue
            o_grid.add(cand[k])
            taken.append(a)
            out.append(mol)
        max_tries -= 1
        if max_tries <= 0:
            raise RuntimeError("water insertion did not converge")
    return np.concatenate(out, 0) if out else np.zeros((0, 3))


def water_box(n_water: int, L: float, seed: int) -> System:
    """``n_water`` waters at random positions and orientations in a cubic box of edge L."""
    rng = np.random.default_rng(seed)
    xyz = _insert_waters(rng, L, n_water)
    types = np.tile(np.array([0, 1, 1], dtype=np.int32), n_water)
    return System(coords=xyz % L, types=types, box=np.diag([L, L, L]).astype(float),
                  n_water=n_water)


def _chain_types(rng, n_chain):
    total = sum(w for _, w in CHAIN_RATIO)
    counts = [int(round(n_chain * w / total)) for _, w in CHAIN_RATIO]
    counts[3] += n_chain - sum(counts)  # absorb rounding into H
    t = np.concatenate([np.full(c, TYPE_INDEX[n], dtype=np.int32) for (n, _), c in zip(CHAIN_RATIO, counts)])
    rng.shuffle(t)
    return t


def _chain_walk(rng, n_chain, L):
    grid = _Grid(L, CHAIN_NONBONDED_MIN)
    pts = [np.full(3, L / 2)]
    grid.add(pts[0])
    while len(pts) < n_chain:
        placed = False
        for _ in range(200):
            b = rng.uniform(1.0, 1.5)
            v = rng.normal(size=3)
            v /= np.linalg.norm(v)
            p = pts[-1] + b * v
            # non-bonded: every earlier chain atom except the predecessor
            if _only_predecessor_close(grid, p, pts[-1]):
                pts.append(p)
                grid.add(p)
                placed = True
                break
        if not placed:
            if len(pts) > 1:
                last = pts.pop()
                bucket = grid.buckets[grid._key(last)]
                for idx in range(len(bucket)):
                    if np.array_equal(bucket[idx], last):
                        bucket.pop(idx)
                        break
    return np.array(pts)


def _only_predecessor_close(grid: _Grid, p, prev) -> bool:
    """True when every chain atom within the non-bonded limit of p is the predecessor itself."""
    cx, cy, cz = grid._key(p)
    n = grid.n
    reach = int(math.ceil(CHAIN_NONBONDED_MIN / grid.cell))
    seen = set()
    for ox in range(-reach, reach + 1):
        for oy in range(-reach, reach + 1):
            for oz in range(-reach, reach + 1):
                key = ((cx + ox) % n, (cy + oy) % n, (cz + oz) % n)
                if key in seen:
                    continue
                seen.add(key)
                for q in grid.buckets.get(key, ()):
                    d = q - p
                    d -= grid.L * np.rint(d / grid.L)
                    if d @ d < CHAIN_NONBONDED_MIN ** 2 and not np.array_equal(q, prev):
                        return False
    return True


def solvated_chain(n_target: int, n_chain: int, seed: int) -> System:
    """A seeded chain of ``n_chain`` atoms solvated with water to about ``n_target`` atoms at 1 g/cm^3."""
    rng = np.random.default_rng(seed)
    ctypes_ = _chain_types(rng, n_chain)
    n_water = int(round((n_target - n_chain) / 3))
    mass = float(MASSES[ctypes_].sum()) + n_water * WATER_MASS
    L = (mass / DENSITY_AMU_PER_A3) ** (1.0 / 3.0)
    chain = _chain_walk(rng, n_chain, L)
    cgrid = _Grid(L, CHAIN_WATER_MIN)
    for p in chain:
        cgrid.add(p)
    water = _insert_waters(rng, L, n_water, chain_grid=cgrid)
    xyz = np.concatenate([chain, water], 0) % L
    types = np.concatenate([ctypes_, np.tile(np.array([0, 1, 1], dtype=np.int32), n_water)])
    return System(coords=xyz, types=types.astype(np.int32), box=np.diag([L, L, L]).astype(float),
                  n_chain=n_chain, n_water=n_water)


def config_system(name: str) -> System:
    """The named synthetic workloads.

    * ``water192``: 64 H2O in a 12.42 A cubic box (system seed 0);
    * ``chain10k``: 600-atom chain + 3,133 H2O = 9,999 atoms (seed 1);
    * ``chain25k``: 1,200-atom chain + 7,933 H2O = 24,999 atoms (seed 2);
    * ``chain40k``: 2,000-atom chain + 12,667 H2O = 40,001 atoms (seed 3).
    Smaller solvated chains for fast parity runs: ``chain1k`` (seed 11) and ``chain3k`` (seed 12).
    """
    if name == "water192":
        return water_box(64, 12.42, seed=0)
    table = {
        "chain1k": (1000, 60, 11),
        "chain3k": (3000, 180, 12),
        "chain10k": (9999, 600, 1),
        "chain25k": (24999, 1200, 2),
        "chain40k": (40001, 2000, 3),
    }
    if name not in table:
        raise KeyError(name)
    n, nc, seed = table[name]
    return solvated_chain(n, nc, seed)


def request_system(natoms: int, kind: str, seed: int) -> System:
    """One serving request: a water box of natoms//3 molecules or a solvated chain of length round(0.05 N)."""
    if kind == "water":
        n_w = max(1, natoms // 3)
        L = (n_w * WATER_MASS / DENSITY_AMU_PER_A3) ** (1.0 / 3.0)
        return water_box(n_w, L, seed)
    nc = max(2, int(round(0.05 * natoms)))
    return solvated_chain(natoms, nc, seed)


def serving_trace(n_requests: int, rate_per_s: float = 200.0, seed: int = 4,
                  n_min: int = 192, n_max: int = 40000):
    """Poisson arrivals; sizes log-uniform in [n_min, n_max]; a seeded coin picks water box or chain.

    Returns a list of dicts: arrival time (s), natoms, kind, system seed.
    """
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate_per_s, size=n_requests))
    sizes = np.round(np.exp(rng.uniform(math.log(n_min), math.log(n_max), size=n_requests))).astype(int)
    kinds = np.where(rng.random(n_requests) < 0.5, "water", "chain")
    seeds = rng.integers(1000, 2**31 - 1, size=n_requests)
    return [dict(t=float(a), natoms=int(n), kind=str(k), seed=int(s))
            for a, n, k, s in zip(t, sizes, kinds, seeds)]
