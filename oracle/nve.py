"""Velocity-Verlet NVE driver on the oracle's forces (for the energy-drift check).

Units: A, fs, amu, eV.  1 eV/(A amu) = 9.648533e-3 A/fs^2.  Maxwell-Boltzmann
velocities at temperature T with the centre-of-mass momentum removed.
"""
from __future__ import annotations

import numpy as np

from .dp import evaluate

ACC = 9.648533e-3          # (eV/A)/amu -> A/fs^2
KB = 8.617333262e-5        # eV/K
MASSES = np.array([15.999, 1.008, 12.011, 14.007, 32.06])


def maxwell_boltzmann(types, T: float, seed: int):
    rng = np.random.default_rng(seed)
    m = MASSES[types]
    v = rng.normal(size=(len(types), 3)) * np.sqrt(KB * T * ACC / m)[:, None]
    v -= (m[:, None] * v).sum(0) / m.sum()
    return v


def kinetic(types, v):
    m = MASSES[types]
    return 0.5 * float((m[:, None] * v * v).sum()) / ACC


def run_nve(model, X, types, box, v, dt: float, steps: int):
    """Returns the total energy after each step (index 0 = initial)."""
    return run_nve_traj(model, X, types, box, v, dt, steps)[0]


def run_nve_traj(model, X, types, box, v, dt: float, steps: int):
    """Total energy after each step (index 0 = initial), final positions and velocities."""
    X = np.array(X, dtype=np.float64)
    v = np.array(v, dtype=np.float64)
    inv_m = (ACC / MASSES[types])[:, None]
    out = evaluate(model, X, types, box)
    F = out["F"]
    etot = [out["E"] + kinetic(types, v)]
    for _ in range(steps):
        v += 0.5 * dt * F * inv_m
        X += dt * v
        out = evaluate(model, X, types, box)
        F = out["F"]
        v += 0.5 * dt * F * inv_m
        etot.append(out["E"] + kinetic(types, v))
    return np.array(etot), X, v
