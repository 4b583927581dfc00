"""Seeded synthetic geometries standing in for the paper's workloads.

The paper's own structures (the 53-atom lig_30 ligand, the GFP chromophore in
167 waters, CDK8 in 41,194 waters) are not available, so these generators give
inputs of the same kind: small organic-density molecules, batches of
conformations, and liquid-density water boxes.  Positions are generated in
float64 and cast once to float32; the float32 values are canonical.
"""
from __future__ import annotations

from dataclasses import dataclass
import numpy as np

from .params import SPECIES7

SPECIES7_WEIGHTS = np.array([0.45, 0.3, 0.1, 0.1, 0.02, 0.02, 0.01])


@dataclass
class System:
    pos: np.ndarray          # float32 [N, 3], Angstrom
    species: np.ndarray      # int32 [N]
    mol_offsets: np.ndarray  # int32 [n_mol + 1]
    box: np.ndarray | None   # float32 [3] orthorhombic edge lengths, or None
    n_species: int
    name: str = ""

    @property
    def n_atoms(self) -> int:
        return int(self.pos.shape[0])

    @property
    def n_mol(self) -> int:
        return int(self.mol_offsets.shape[0] - 1)

    def molecule(self, m: int) -> "System":
        a, b = int(self.mol_offsets[m]), int(self.mol_offsets[m + 1])
        return System(self.pos[a:b].copy(), self.species[a:b].copy(),
                      np.array([0, b - a], dtype=np.int32), self.box, self.n_species,
                      f"{self.name}[{m}]")


def random_molecule(n_atoms: int, side: float, min_sep: float, rng) -> np.ndarray:
    """Uniform positions in [0, side)^3 by sequential rejection so that every
    pair is at least ``min_sep`` apart (float64)."""
    pts = np.empty((n_atoms, 3))
    k = 0
    tries = 0
    while k < n_atoms:
        p = rng.uniform(0.0, side, 3)
        tries += 1
        if tries > 1000000:
            raise RuntimeError("rejection sampling did not converge")
        if k and np.min(np.sum((pts[:k] - p) ** 2, axis=1)) < min_sep * min_sep:
            continue
        pts[k] = p
        k += 1
    return pts


def draw_species(n: int, n_species: int, rng) -> np.ndarray:
    if n_species == 4:
        return rng.integers(0, 4, n).astype(np.int32)
    w = SPECIES7_WEIGHTS / SPECIES7_WEIGHTS.sum()
    return rng.choice(len(SPECIES7), size=n, p=w).astype(np.int32)


def single_molecule(n_atoms: int = 24, seed: int = 0, n_species: int = 4,
                    side: float | None = None) -> System:
    """Config 0 procedure: side 10 A at 24 atoms, scaled to constant density."""
    rng = np.random.default_rng(seed)
    if side is None:
        side = 10.0 * (n_atoms / 24.0) ** (1.0 / 3.0)
    sp = draw_species(n_atoms, n_species, rng)
    pos = random_molecule(n_atoms, side, 0.9, rng)
    return System(pos.astype(np.float32), sp, np.array([0, n_atoms], np.int32), None,
                  n_species, f"mol{n_atoms}")


def conformer_batch(n_conf: int = 512, n_atoms: int = 64, seed: int = 1,
                    jitter: float = 0.05, n_species: int = 7) -> System:
    """Config 1: ``n_conf`` jittered copies of one random molecule."""
    base = single_molecule(n_atoms, seed, n_species)
    rng = np.random.default_rng(seed + 1000)
    pos = base.pos.astype(np.float64)[None] + rng.normal(0.0, jitter, (n_conf, n_atoms, 3))
    return System(pos.reshape(-1, 3).astype(np.float32),
                  np.tile(base.species, n_conf).astype(np.int32),
                  (np.arange(n_conf + 1) * n_atoms).astype(np.int32), None, n_species,
                  f"batch{n_conf}x{n_atoms}")


def _random_rotations(n: int, rng) -> np.ndarray:
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)], -1),
        np.stack([2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)], -1),
        np.stack([2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)], -1),
    ], 1)


def _rsa_points(n: int, L: float, dmin: float, rng) -> np.ndarray:
    """Random sequential addition in a periodic cube, grid-accelerated: each
    candidate is tested against the points already placed in its 27
    surrounding grid cells (cells at least ``dmin`` wide)."""
    nc = max(3, int(L // dmin))
    cell = L / nc
    cap = 16
    grid = np.full((nc, nc, nc, cap), -1, dtype=np.int64)
    fill = np.zeros((nc, nc, nc), dtype=np.int64)
    pts = np.zeros((n + 1, 3))
    pts[n] = 1e9  # sentinel for empty slots: never within dmin
    off = np.array([(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)])
    k = 0
    d2 = dmin * dmin
    tries = 0
    while k < n:
        cand = rng.uniform(0.0, L, (1024, 3))
        cells = np.minimum((cand // cell).astype(np.int64), nc - 1)
        for p, c in zip(cand, cells):
            tries += 1
            nb = (c[None, :] + off) % nc
            idx = grid[nb[:, 0], nb[:, 1], nb[:, 2]].ravel()
            idx = np.where(idx < 0, n, idx)
            q = pts[idx] - p
            q -= L * np.rint(q / L)
            if np.min((q * q).sum(1)) < d2:
                continue
            f = fill[c[0], c[1], c[2]]
            if f >= cap:
                continue
            pts[k] = p
            grid[c[0], c[1], c[2], f] = k
            fill[c[0], c[1], c[2]] = f + 1
            k += 1
            if k == n:
                break
        if tries > 200 * n + 100000:
            raise RuntimeError("RSA did not reach the requested density")
    return pts[:n]


def water_box(n_water: int, L: float, seed: int, n_species: int = 4) -> System:
    """Rigid-geometry waters (O-H 0.9572 A, H-O-H 104.52 deg) with random
    orientations; O-O min-image distance >= 2.6 A; atom order O, H, H;
    positions wrapped into [0, L)."""
    rng = np.random.default_rng(seed)
    O = _rsa_points(n_water, L, 2.6, rng)
    R = _random_rotations(n_water, rng)
    half = np.deg2rad(104.52) / 2.0
    h1 = 0.9572 * np.array([np.sin(half), 0.0, np.cos(half)])
    h2 = 0.9572 * np.array([-np.sin(half), 0.0, np.cos(half)])
    H1 = O + R @ h1
    H2 = O + R @ h2
    pos = np.stack([O, H1, H2], 1).reshape(-1, 3)
    pos = np.mod(pos, L).astype(np.float32)
    pos[pos >= np.float32(L)] = 0.0
    sp = np.tile(np.array([3, 0, 0], np.int32), n_water)
    return System(pos, sp, np.array([0, 3 * n_water], np.int32),
                  np.full(3, L, np.float32), n_species, f"water{n_water}")


def triclinic_system(n_atoms: int, box, seed: int = 0, n_species: int = 4,
                     min_sep: float = 0.9) -> System:
    """Atoms uniform in a triclinic cell (rows a, b, c of ``box``), placed by
    sequential rejection at a minimum-image separation of ``min_sep``; the
    positions are wrapped into the cell (fractional coordinates in [0, 1))."""
    rng = np.random.default_rng(seed)
    B = np.asarray(box, dtype=np.float64)
    pts = np.empty((n_atoms, 3))
    k = 0
    tries = 0
    while k < n_atoms:
        tries += 1
        if tries > 1000000:
            raise RuntimeError("rejection sampling did not converge")
        p = rng.uniform(0.0, 1.0, 3) @ B
        if k:
            d = pts[:k] - p
            for r in (2, 1, 0):
                d = d - np.rint(d[:, r] / B[r, r])[:, None] * B[r]
            if np.min(np.sum(d * d, axis=1)) < min_sep * min_sep:
                continue
        pts[k] = p
        k += 1
    sp = draw_species(n_atoms, n_species, rng)
    return System(pts.astype(np.float32), sp, np.array([0, n_atoms], np.int32),
                  np.asarray(box, dtype=np.float32), n_species, f"triclinic{n_atoms}")


def config_system(k: int, **kw) -> System:
    """The synthetic system of workload k (0: 24-atom molecule; 1: 512x64
    conformations; 2: 1,500-water box; 3: a packed batch of serving-sized
    molecules; 4: 7,667-water box)."""
    if k == 0:
        return single_molecule(24, seed=0, n_species=4)
    if k == 1:
        return conformer_batch(kw.get("n_conf", 512), 64, seed=1)
    if k == 2:
        return water_box(1500, 35.5, seed=2, n_species=4)
    if k == 3:
        from .requests import poisson_requests
        reqs = poisson_requests(kw.get("n_req", 32), rate=1.0, seed=3)
        return pack_molecules([r.system for r in reqs], 7, "serving-batch")
    if k == 4:
        return water_box(7667, 61.2, seed=4, n_species=7)
    raise ValueError(k)


def pack_molecules(mols, n_species: int, name: str = "") -> System:
    pos = np.concatenate([m.pos for m in mols]).astype(np.float32)
    sp = np.concatenate([m.species for m in mols]).astype(np.int32)
    off = np.concatenate([[0], np.cumsum([m.n_atoms for m in mols])]).astype(np.int32)
    return System(pos, sp, off, None, n_species, name)


CONFIGS = {
    0: "24-atom molecule, 4 species, no PBC",
    1: "512 conformations x 64 atoms, 7 species, no PBC",
    2: "1,500-water box (4,500 atoms), L=35.5 A, 4 species",
    3: "serving stream, molecules of 10-150 atoms, 7 species",
    4: "7,667-water box (23,001 atoms), L=61.2 A, 7 species",
}
