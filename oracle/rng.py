"""Counter-based random numbers for the Langevin integrator (oracle; test
use only).

Philox4x32-10 as published by Salmon, Moraes, Dror and Shaw, "Parallel random
numbers: as easy as 1, 2, 3" (SC '11): a 128-bit counter and a 64-bit key;
ten rounds, each multiplying counter words 0 and 2 by fixed odd constants
into 64-bit products, then mixing the high halves with words 1 and 3 and the
key; the key is bumped by two Weyl constants between rounds.  Written here
with Python integers (exact), one block at a time.

Normal deviates come from the Box-Muller transform in float64 over pairs of
32-bit outputs: u = (w + 1) / 2^32 in (0, 1], theta = 2 pi w' / 2^32,
n = sqrt(-2 ln u) (cos theta, sin theta).

The counter layout used by the integrator (an interface both sides agree
on): counter = (atom index, step mod 2^32, step div 2^32, 0), key = (seed mod
2^32, seed div 2^32); the first three normals of the block drive the atom's
three velocity components.
"""
from __future__ import annotations

import math

import numpy as np

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9  # golden ratio
W1 = 0xBB67AE85  # sqrt(3) - 1
MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """One Philox4x32 block with 10 rounds: 4 counter words, 2 key words ->
    4 output words (Python ints)."""
    c0, c1, c2, c3 = (int(x) & MASK for x in ctr)
    k0, k1 = (int(x) & MASK for x in key)
    for r in range(10):
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = p0 >> 32, p0 & MASK
        hi1, lo1 = p1 >> 32, p1 & MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
        if r < 9:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
    return c0, c1, c2, c3


def box_muller(wa, wb):
    u = (wa + 1) * 2.0 ** -32
    th = 2.0 * math.pi * wb * 2.0 ** -32
    r = math.sqrt(-2.0 * math.log(u))
    return r * math.cos(th), r * math.sin(th)


def atom_normals(i, step, seed):
    """The three standard normals of atom i at integrator step `step`."""
    w = philox4x32_10((i, step & MASK, step >> 32, 0), (seed & MASK, seed >> 32))
    n0, n1 = box_muller(w[0], w[1])
    n2, _ = box_muller(w[2], w[3])
    return n0, n1, n2


def normals(n_atoms, step, seed):
    return np.array([atom_normals(i, step, seed) for i in range(n_atoms)], dtype=np.float64)
