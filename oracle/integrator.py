"""Velocity-Verlet molecular dynamics, float64 state (oracle; test use only).

Units: A, fs, amu, eV.  An acceleration is a = 9.648533e-3 * F / m A/fs^2
(1 eV/A/amu = 9.648533e-3 A/fs^2) and the kinetic energy is
KE = 0.5 * sum m v^2 / 9.648533e-3 eV.  Positions and velocities are float64;
forces are evaluated at the float32 rounding of the positions, as the
potential's inputs are float32.

One step:  v += (dt/2) a(x);  x += dt v;  v += (dt/2) a(x_new).

``langevin_middle`` is the LF-Middle Langevin scheme (NVT), with normals from
the counter-based generator in ``rng``.
"""
from __future__ import annotations

import math

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


KB_EV = 8.617333262e-5  # Boltzmann constant, eV/K


def langevin_middle(x0, v_half0, masses, force_fn, dt, n_steps, temperature, friction_per_ps,
                    seed, step0: int = 0, record_every: int = 1):
    """LF-Middle Langevin dynamics (Methods, "Other Features": the LF-Middle
    discretization OpenMM added; Results, GFP example: NVT at 300 K, 0.5 fs,
    1 / ps).  A leapfrog scheme with the thermostat between two half drifts;
    velocities live at half steps.  One step, from x_n, v_{n-1/2} and F(x_n):

        v <- v + dt a(x_n)
        x <- x + dt/2 v
        v <- c v + sqrt((1 - c^2) kT / m) R,   c = exp(-friction dt)
        x <- x + dt/2 v                        (= x_{n+1}; v = v_{n+1/2})

    R are standard normals from ``rng.atom_normals(i, step0 + n, seed)``.
    kT/m is a velocity variance in A^2/fs^2: kB T * ACC_UNIT / m.  Records
    hold (step, E_pot(x_n), KE of v_{n-1/2})."""
    from .rng import normals
    x = np.array(x0, dtype=np.float64)
    v = np.array(v_half0, dtype=np.float64)
    m = np.asarray(masses, dtype=np.float64)[:, None]
    c = math.exp(-friction_per_ps * 1e-3 * dt)
    sig = np.sqrt((1.0 - c * c) * KB_EV * temperature * ACC_UNIT / m)
    E, F = force_fn(x.astype(np.float32))
    rec = [(0, float(np.sum(E)), float(kinetic_energy(v, m[:, 0])))]
    for n in range(n_steps):
        v = v + dt * ACC_UNIT * F / m
        x = x + 0.5 * dt * v
        v = c * v + sig * normals(x.shape[0], step0 + n, seed)
        x = x + 0.5 * dt * v
        E, F = force_fn(x.astype(np.float32))
        if (n + 1) % record_every == 0 or n + 1 == n_steps:
            rec.append((n + 1, float(np.sum(E)), float(kinetic_energy(v, m[:, 0]))))
    return x, v, rec
