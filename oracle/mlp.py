"""Per-element atomic networks, float64 (oracle; test use only).

ANI potentials give every element its own feed-forward network and sum the
atomic outputs to the molecular energy (Methods, "OpenMM-ML": seven elements
for ANI-2x, four for ANI-1ccx).  Hidden layers use
CELU_alpha(x) = max(0, x) + min(0, alpha (exp(x / alpha) - 1)):

  h_0 = G_i;  h_l = CELU(W_l h_(l-1) + b_l), l = 1..L-1;
  E_i = W_L h_(L-1) + b_L            (W, b of the element of atom i).

The adjoint is ordinary backpropagation: delta_L = dE/dE_i,
delta_l = (W_(l+1)^T delta_(l+1)) * CELU'(z_l), dE/dG_i = W_1^T delta_1,
dE/dW_l = sum_i delta_l,i h_(l-1),i^T, dE/db_l = sum_i delta_l,i.
"""
from __future__ import annotations

import numpy as np


def celu(x, alpha):
    x = np.asarray(x, dtype=np.float64)
    return np.maximum(x, 0.0) + np.minimum(0.0, alpha * np.expm1(np.minimum(x, 0.0) / alpha))


def celu_grad(x, alpha):
    x = np.asarray(x, dtype=np.float64)
    return np.where(x > 0.0, 1.0, np.exp(np.minimum(x, 0.0) / alpha))


def _params64(table, s):
    return ([w.astype(np.float64) for w in table.W[s]],
            [b.astype(np.float64) for b in table.b[s]])


def mlp_forward(G, species, table):
    """Atomic energies E_i [N] (without self energies) and the activations."""
    G = np.asarray(G, dtype=np.float64)
    sp = np.asarray(species)
    N = G.shape[0]
    E = np.zeros(N)
    cache = {}
    alpha = table.celu_alpha
    L = table.n_layers
    for s in range(table.n_species):
        rows = np.nonzero(sp == s)[0]
        if rows.size == 0:
            continue
        W, b = _params64(table, s)
        h = G[rows]
        hs, zs = [h], []
        for l in range(L):
            z = h @ W[l].T + b[l]
            zs.append(z)
            if l < L - 1:
                h = celu(z, alpha)
                hs.append(h)
        E[rows] = zs[-1][:, 0]
        cache[s] = (rows, hs, zs)
    return E, cache


def _deltas(cache_s, W, dE_rows, alpha):
    rows, hs, zs = cache_s
    L = len(W)
    deltas = [None] * L
    deltas[L - 1] = dE_rows[:, None]                     # d E / d z_L
    for l in range(L - 2, -1, -1):
        deltas[l] = (deltas[l + 1] @ W[l + 1]) * celu_grad(zs[l], alpha)
    return deltas


def mlp_backward_input(cache, dE_atom, table):
    """dE/dG [N, F] given upstream dE/dE_i [N]."""
    dE_atom = np.asarray(dE_atom, dtype=np.float64)
    N = dE_atom.shape[0]
    F = table.widths[0]
    g = np.zeros((N, F))
    for s, cs in cache.items():
        W, _ = _params64(table, s)
        rows = cs[0]
        d = _deltas(cs, W, dE_atom[rows], table.celu_alpha)
        g[rows] = d[0] @ W[0]
    return g


def mlp_weight_grads(cache, dE_atom, table):
    """(dW[s][l], db[s][l]) in float64 given upstream dE/dE_i [N]."""
    dE_atom = np.asarray(dE_atom, dtype=np.float64)
    dW = [[np.zeros(w.shape) for w in table.W[s]] for s in range(table.n_species)]
    db = [[np.zeros(b.shape) for b in table.b[s]] for s in range(table.n_species)]
    for s, cs in cache.items():
        W, _ = _params64(table, s)
        rows, hs, _zs = cs
        d = _deltas(cs, W, dE_atom[rows], table.celu_alpha)
        for l in range(table.n_layers):
            dW[s][l] = d[l].T @ hs[l]
            db[s][l] = d[l].sum(0)
    return dW, db
