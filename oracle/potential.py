"""Energy per molecule, analytic forces and weight gradients, float64
(oracle; test use only).

E_m = sum over atoms i of molecule m of (E_i + e_self[s_i]); forces are
F = -dE/dr, obtained by backpropagating through the networks and the
symmetry functions (the paper's TorchForce contract: a model maps positions to
energy and forces follow by backpropagation, Methods "PyTorch Model
Support").  Molecules are independent: there are no cross-molecule pairs.
"""
from __future__ import annotations

from dataclasses import dataclass
import numpy as np

from .aev import aev, aev_backward, n_features
from .mlp import mlp_forward, mlp_backward_input, mlp_weight_grads


@dataclass
class EFResult:
    E: np.ndarray          # float64 [n_mol]
    F: np.ndarray | None   # float64 [N, 3]
    E_atom: np.ndarray     # float64 [N] (network output, no self energy)
    G: np.ndarray          # float64 [N, F]


def _mol_index(mol_offsets, N):
    off = np.asarray(mol_offsets, dtype=np.int64)
    mol = np.zeros(N, dtype=np.int64)
    for m in range(off.shape[0] - 1):
        mol[off[m]:off[m + 1]] = m
    return mol


def _check(species, aev_t, mlp_t):
    S = aev_t.n_species
    if mlp_t.n_species != S:
        raise ValueError("species count of the AEV table and the networks differ")
    if mlp_t.widths[0] != n_features(S, aev_t.n_r, aev_t.n_a, aev_t.n_z):
        raise ValueError("first layer width does not match the AEV length")
    sp = np.asarray(species)
    if sp.size and (sp.min() < 0 or sp.max() >= S):
        raise ValueError("species index out of range")


def energy_forces(sys_or_pos, species=None, mol_offsets=None, box=None, *,
                  aev_table, mlp_table, forces: bool = True, pairs=None) -> EFResult:
    """Energies and forces.  ``pairs`` = (radial pairs, angular pairs) fixes
    the neighbor sets (used when positions are perturbed in float64)."""
    if species is None:
        s = sys_or_pos
        pos, species, mol_offsets, box = s.pos, s.species, s.mol_offsets, s.box
    else:
        pos = sys_or_pos
    _check(species, aev_table, mlp_table)
    N = pos.shape[0]
    mol = _mol_index(mol_offsets, N)
    n_mol = len(mol_offsets) - 1
    pr, pa = pairs if pairs is not None else (None, None)
    G, ac = aev(pos, species, mol_offsets, box, aev_table, pr, pa)
    Ea, mc = mlp_forward(G, species, mlp_table)
    Etot = Ea + mlp_table.self_energy[np.asarray(species)]
    E = np.bincount(mol, weights=Etot, minlength=n_mol)
    F = None
    if forces:
        g = mlp_backward_input(mc, np.ones(N), mlp_table)
        F = -aev_backward(g, ac)
    return EFResult(E, F, Ea, G)


def energy(pos, species, mol_offsets, box, aev_table, mlp_table, pairs=None):
    return energy_forces(pos, species, mol_offsets, box, aev_table=aev_table,
                         mlp_table=mlp_table, forces=False, pairs=pairs).E


def weight_gradients(sys_or_pos, species=None, mol_offsets=None, box=None, *,
                     aev_table, mlp_table, dL_dE=None):
    """dL/dtheta as one float64 vector in ``MLPTable.flat`` order, for
    L = sum_m dL_dE[m] * E_m (dL_dE defaults to all ones), plus dL/dpos."""
    if species is None:
        s = sys_or_pos
        pos, species, mol_offsets, box = s.pos, s.species, s.mol_offsets, s.box
    else:
        pos = sys_or_pos
    _check(species, aev_table, mlp_table)
    N = pos.shape[0]
    mol = _mol_index(mol_offsets, N)
    n_mol = len(mol_offsets) - 1
    w = np.ones(n_mol) if dL_dE is None else np.asarray(dL_dE, dtype=np.float64)
    G, ac = aev(pos, species, mol_offsets, box, aev_table)
    _Ea, mc = mlp_forward(G, species, mlp_table)
    up = w[mol]
    dW, db = mlp_weight_grads(mc, up, mlp_table)
    parts = []
    for s in range(mlp_table.n_species):
        for l in range(mlp_table.n_layers):
            parts.append(dW[s][l].ravel())
            parts.append(db[s][l].ravel())
    g = mlp_backward_input(mc, up, mlp_table)
    dpos = aev_backward(g, ac)
    return np.concatenate(parts), dpos


def ensemble_energy_forces(sys_or_pos, species=None, mol_offsets=None, box=None, *,
                           aev_table, mlp_tables, forces: bool = True) -> EFResult:
    """Ensemble of independently trained networks over one set of symmetry
    functions (Results, "Performance of MLPs": ANI-2x averages eight models,
    Table 3 times the ensemble against a single member).  The ensemble energy
    is the mean of the members' energies, so its forces are the mean of the
    members' forces; by linearity the adjoint of the symmetry functions is
    applied once, to the mean of the members' dE/dG.  Self energies are the
    first member's (members share them)."""
    if species is None:
        s = sys_or_pos
        pos, species, mol_offsets, box = s.pos, s.species, s.mol_offsets, s.box
    else:
        pos = sys_or_pos
    M = len(mlp_tables)
    if M < 1:
        raise ValueError("an ensemble needs at least one member")
    for t in mlp_tables:
        _check(species, aev_table, t)
    N = pos.shape[0]
    mol = _mol_index(mol_offsets, N)
    n_mol = len(mol_offsets) - 1
    G, ac = aev(pos, species, mol_offsets, box, aev_table)
    Ea = np.zeros(N)
    g = None
    for t in mlp_tables:
        Ea_k, mc = mlp_forward(G, species, t)
        Ea += Ea_k
        if forces:
            g_k = mlp_backward_input(mc, np.ones(N), t)
            g = g_k if g is None else g + g_k
    Ea /= M
    Etot = Ea + mlp_tables[0].self_energy[np.asarray(species)]
    E = np.bincount(mol, weights=Etot, minlength=n_mol)
    F = None
    if forces:
        F = -aev_backward(g / M, ac)
    return EFResult(E, F, Ea, G)


def subset_energy_forces(pos_all, idx, species, mol_offsets, box=None, *, aev_table,
                         mlp_table, F_other=None):
    """The potential on a subset of a larger system (Results, "Performance
    of MLPs": a ligand modelled by the network inside a classically modelled
    system; mechanical embedding, so the network sees only the subset).
    Subset atom i is row idx[i] of ``pos_all``; ``species`` and
    ``mol_offsets`` are subset-local.  Returns the subset's molecular
    energies and the full-system force array: ``F_other`` (zeros if None)
    plus the subset's forces added at rows idx."""
    idx = np.asarray(idx, dtype=np.int64)
    pos_all = np.asarray(pos_all)
    if idx.size != np.unique(idx).size:
        raise ValueError("subset rows must be distinct")
    r = energy_forces(pos_all[idx], species, mol_offsets, box, aev_table=aev_table,
                      mlp_table=mlp_table)
    F = np.zeros(pos_all.shape, dtype=np.float64) if F_other is None else \
        np.array(F_other, dtype=np.float64)
    F[idx] += r.F
    return r.E, F
