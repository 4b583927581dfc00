"""Serving workload: a Poisson stream of short MD requests on small molecules.

Sizes are log-uniform on 10..150 atoms; geometry follows the single-molecule
procedure at constant density; species use the seven-element weights;
velocities are Maxwell-Boltzmann at 300 K with the centre-of-mass velocity
removed per molecule.  Units: A, fs, amu, eV.
"""
from __future__ import annotations

from dataclasses import dataclass
import numpy as np

from .geometry import System, single_molecule
from .params import MASS_AMU

KB_EV = 8.617333262e-5      # Boltzmann constant, eV/K
EV_TO_AMU_A2_FS2 = 9.648533e-3  # 1 eV = 9.648533e-3 amu A^2 / fs^2


@dataclass
class Request:
    req_id: int
    t_arrive: float       # seconds from stream start
    system: System
    vel: np.ndarray       # float64 [N, 3], A/fs
    n_steps: int


def maxwell_boltzmann(species: np.ndarray, T: float, rng) -> np.ndarray:
    m = MASS_AMU[species]
    sigma = np.sqrt(KB_EV * T * EV_TO_AMU_A2_FS2 / m)
    v = rng.standard_normal((species.shape[0], 3)) * sigma[:, None]
    vcm = (m[:, None] * v).sum(0) / m.sum()
    return v - vcm


def request_sizes(n: int, rng, lo: int = 10, hi: int = 150) -> np.ndarray:
    return np.floor(np.exp(rng.uniform(np.log(lo), np.log(hi + 1), n))).astype(int)


def poisson_requests(n: int, rate: float, seed: int = 3, arrival_seed: int = 30,
                     n_steps: int = 100, T: float = 300.0) -> list:
    """``n`` requests arriving at ``rate`` per second (exponential gaps)."""
    rng = np.random.default_rng(seed)
    arr = np.random.default_rng(arrival_seed)
    t = np.cumsum(arr.exponential(1.0 / rate, n))
    sizes = request_sizes(n, rng)
    out = []
    for i in range(n):
        mol = single_molecule(int(sizes[i]), seed=int(rng.integers(1 << 30)), n_species=7)
        v = maxwell_boltzmann(mol.species, T, rng)
        out.append(Request(i, float(t[i]), mol, v, n_steps))
    return out
