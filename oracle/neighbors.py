"""Neighbor sets under the float32 distance predicate (oracle; test use only).

The paper lists neighbor-list construction among the bottleneck operations it
accelerates (Methods, "Optimization Through NNPOps") but does not define the
predicate.  The reading used here makes pair sets reproducible bit for bit:

* displacement per component  dx = fl32(x_j - x_i); with an orthorhombic box
  of edge L, dx = fl32(dx - fl32(L * rint(fl32(dx * invL)))), invL = fl32(1/L),
  rint rounding half to even (minimum image);
* a triclinic box is given by its row vectors a = (ax, 0, 0),
  b = (bx, by, 0), c = (cx, cy, cz) in reduced form (ax, by, cz > 0,
  |bx|, |cx| <= ax/2, |cy| <= by/2); the image is removed along c, then b,
  then a, each step n = rint(fl32(d_k * fl32(1/v_kk))) and
  d -= fl32(v * n) component by component (k = z, y, x).  With the cutoff at
  most half of every perpendicular width this is the minimum image;
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


def is_triclinic(box) -> bool:
    return box is not None and np.asarray(box).shape == (3, 3)


def check_triclinic(box, rc) -> None:
    """Raise ValueError unless ``box`` is a reduced triclinic cell whose
    perpendicular widths are all at least 2 rc."""
    v = np.asarray(box, dtype=np.float64)
    ax, by, cz = v[0, 0], v[1, 1], v[2, 2]
    if v[0, 1] != 0 or v[0, 2] != 0 or v[1, 2] != 0 or min(ax, by, cz) <= 0:
        raise ValueError("box rows must be a=(ax,0,0), b=(bx,by,0), c=(cx,cy,cz)")
    if abs(v[1, 0]) > ax / 2 or abs(v[2, 0]) > ax / 2 or abs(v[2, 1]) > by / 2:
        raise ValueError("box is not in reduced form")
    if min(perpendicular_widths(v)) < 2 * rc:
        raise ValueError("box narrower than twice the cutoff")


def perpendicular_widths(box):
    v = np.asarray(box, dtype=np.float64)
    vol = abs(np.linalg.det(v))
    return [vol / np.linalg.norm(np.cross(v[1], v[2])),
            vol / np.linalg.norm(np.cross(v[2], v[0])),
            vol / np.linalg.norm(np.cross(v[0], v[1]))]


def _tric_image(d, box):
    """Reduced-form image removal on float32 component arrays [dx, dy, dz]."""
    v = np.asarray(box, dtype=f32)
    for k in (2, 1, 0):
        inv = f32(f32(1.0) / v[k, k])
        n = np.rint((d[k] * inv).astype(f32)).astype(f32)
        d = [(d[c] - (v[k, c] * n).astype(f32)).astype(f32) if c <= k else d[c]
             for c in range(3)]
    return d


def _d2_rows(pos, i0, i1, a, b, box):
    """float32 d2 between atoms i0..i1 and a..b (rows x cols)."""
    xi = pos[i0:i1]
    xj = pos[a:b]
    comps = []
    tric = is_triclinic(box)
    for c in range(3):
        d = (xj[None, :, c] - xi[:, None, c]).astype(f32)
        if box is not None and not tric:
            L = f32(box[c])
            invL = f32(f32(1.0) / L)
            d = (d - (L * np.rint((d * invL).astype(f32))).astype(f32)).astype(f32)
        comps.append(d)
    if tric:
        comps = _tric_image(comps, box)
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
                dd = [f32(f32(pos32[j, c]) - f32(pos32[i, c])) for c in range(3)]
                if is_triclinic(box):
                    v = np.asarray(box, dtype=f32)
                    for k in (2, 1, 0):
                        n = f32(np.rint(f32(dd[k] * f32(f32(1.0) / v[k, k]))))
                        for c in range(k + 1):
                            dd[c] = f32(dd[c] - f32(v[k, c] * n))
                elif box is not None:
                    for c in range(3):
                        L = f32(box[c])
                        invL = f32(f32(1.0) / L)
                        dd[c] = f32(dd[c] - f32(L * f32(np.rint(f32(dd[c] * invL)))))
                for c in range(3):
                    d = dd[c]
                    d2 = f32(d2 + f32(d * d)) if c else f32(d * d)
                if d2 < rc2:
                    out.append((i, j))
    out.sort()
    if not out:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    a = np.array(out, dtype=np.int64)
    return a[:, 0], a[:, 1]
