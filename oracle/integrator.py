"""Velocity-Verlet molecular dynamics, float64 state (oracle; test use only).

Units: A, fs, amu, eV.  An acceleration is a = 9.648533e-3 * F / m A/fs^2
(1 eV/A/amu = 9.648533e-3 A/fs^2) and the kinetic energy is
KE = 0.5 * sum m v^2 / 9.648533e-3 eV.  Positions and velocities are float64;
forces are evaluated at the float32 rounding of the positions, as the
potential's inputs are float32.

One step:  v += (dt/2) a(x);  x += dt v;  v += (dt/2) a(x_new).
"""
from __future__ import annotations

import numpy as np

ACC_UNIT = 9.648533e-3


def kinetic_energy(v, masses, mol_offsets=None):
    ke = 0.5 * (np.asarray(masses)[:, None] * v * v).sum(1) / ACC_UNIT
    if mol_offsets is None:
        return ke.sum()
    off = np.asarray(mol_offsets)
    return np.array([ke[off[m]:off[m + 1]].sum() for m in range(off.shape[0] - 1)])


def velocity_verlet(x0, v0, masses, force_fn, dt, n_steps, record_every: int = 1):
    """Integrate ``n_steps``.  ``force_fn(pos32) -> (E_pot, F)``.  Returns the
    final (x, v) and a list of (step, E_pot, KE) records."""
    x = np.array(x0, dtype=np.float64)
    v = np.array(v0, dtype=np.float64)
    m = np.asarray(masses, dtype=np.float64)[:, None]
    E, F = force_fn(x.astype(np.float32))
    rec = [(0, float(np.sum(E)), float(kinetic_energy(v, m[:, 0])))]
    for n in range(1, n_steps + 1):
        v = v + 0.5 * dt * ACC_UNIT * F / m
        x = x + dt * v
        E, F = force_fn(x.astype(np.float32))
        v = v + 0.5 * dt * ACC_UNIT * F / m
        if n % record_every == 0 or n == n_steps:
            rec.append((n, float(np.sum(E)), float(kinetic_energy(v, m[:, 0]))))
    return x, v, rec
