"""Neighbor sets under the float32 distance predicate (oracle; test use only).

The paper lists neighbor-list construction among the bottleneck operations it
accelerates (Methods, "Optimization Through NNPOps") but does not define the
predicate.  The reading used here makes pair sets reproducible bit for bit:

* displacement per component  dx = fl32(x_j - x_i); with an orthorhombic box
  of edge L, dx = fl32(dx - fl32(L * rint(fl32(dx * invL)))), invL = fl32(1/L),
  rint rounding half to even (minimum image);
* d2 = fl32(fl32(fl32(dx*dx) + fl32(dy*dy)) + fl32(dz*dz)), left to right,
  never fused;
* j is a neighbor of i iff they are in the same molecule, j != i and
  d2 < fl32(fl32(R) * fl32(R)).

NumPy float32 scalar and array arithmetic is IEEE round-to-nearest and never
contracts to FMA, so it evaluates exactly this predicate.
"""
from __future__ import annotations

import numpy as np

f32 = np.float32


def cutoff_sq(rc) -> np.float32:
    r = f32(rc)
    return f32(r * r)


def _d2_rows(pos, i0, i1, a, b, box):
    """float32 d2 between atoms i0..i1 and a..b (rows x cols)."""
    xi = pos[i0:i1]
    xj = pos[a:b]
    comps = []
    for c in range(3):
        d = (xj[None, :, c] - xi[:, None, c]).astype(f32)
        if box is not None:
            L = f32(box[c])
            invL = f32(f32(1.0) / L)
            d = (d - (L * np.rint((d * invL).astype(f32))).astype(f32)).astype(f32)
        comps.append(d)
    d2 = (comps[0] * comps[0]).astype(f32)
    d2 = (d2 + (comps[1] * comps[1]).astype(f32)).astype(f32)
    d2 = (d2 + (comps[2] * comps[2]).astype(f32)).astype(f32)
    return d2


def pair_list(pos32, mol_offsets, box, rc, chunk: int = 1024):
    """Full (ordered) neighbor list: arrays (i, j), sorted by i then j, of all
    same-molecule pairs with d2 < rc^2 under the float32 predicate."""
    pos = np.ascontiguousarray(pos32, dtype=f32)
    rc2 = cutoff_sq(rc)
    I, J = [], []
    off = np.asarray(mol_offsets)
    for m in range(off.shape[0] - 1):
        a, b = int(off[m]), int(off[m + 1])
        for i0 in range(a, b, chunk):
            i1 = min(b, i0 + chunk)
            d2 = _d2_rows(pos, i0, i1, a, b, box)
            ii, jj = np.nonzero(d2 < rc2)
            ii = ii + i0
            jj = jj + a
            keep = ii != jj
            I.append(ii[keep])
            J.append(jj[keep])
    if not I:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    I = np.concatenate(I).astype(np.int64)
    J = np.concatenate(J).astype(np.int64)
    o = np.lexsort((J, I))
    return I[o], J[o]


def pair_list_loops(pos32, mol_offsets, box, rc):
    """The same predicate as ``pair_list`` evaluated one pair at a time with
    float32 scalars (brute force for tiny inputs)."""
    rc2 = cutoff_sq(rc)
    out = []
    off = [int(x) for x in mol_offsets]
    for m in range(len(off) - 1):
        for i in range(off[m], off[m + 1]):
            for j in range(off[m], off[m + 1]):
                if i == j:
                    continue
                d2 = f32(0.0)
                for c in range(3):
                    d = f32(f32(pos32[j, c]) - f32(pos32[i, c]))
                    if box is not None:
                        L = f32(box[c])
                        invL = f32(f32(1.0) / L)
                        d = f32(d - f32(L * f32(np.rint(f32(d * invL)))))
                    d2 = f32(d2 + f32(d * d)) if c else f32(d * d)
                if d2 < rc2:
                    out.append((i, j))
    out.sort()
    if not out:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    a = np.array(out, dtype=np.int64)
    return a[:, 0], a[:, 1]
