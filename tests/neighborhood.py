"""Oracle reference for one atom of a large periodic system, from its
neighborhood only (test helper; CPU)."""
import numpy as np

import oracle as o
from oracle.neighbors import pair_list


def neighborhood_reference(s, at, mt, k):
    """Atom k's full-system force and radial neighbor set from the oracle on
    its neighborhood.  The force on k depends only on the energies of k and
    its radial neighbors, whose own neighbors lie within 2 R_c of k: the
    oracle on the atoms within 2 R_c + 0.5 A of k (same box, so the same
    minimum-image displacements), with the neighbor lists restricted to
    those centers, gives k's force exactly."""
    rc = at.rc_rad
    box = np.asarray(s.box, np.float64)
    d = s.pos.astype(np.float64) - s.pos[k].astype(np.float64)
    d -= box * np.rint(d / box)
    cl = np.nonzero((d * d).sum(1) < (2 * rc + 0.5) ** 2)[0]
    kl = int(np.nonzero(cl == k)[0][0])
    pos, sp = s.pos[cl], s.species[cl]
    off = np.array([0, cl.size], np.int32)
    pr = pair_list(pos, off, s.box, rc)
    pa = pair_list(pos, off, s.box, at.rc_ang)
    centers = np.zeros(cl.size, bool)
    centers[kl] = True
    centers[pr[1][pr[0] == kl]] = True
    keep_r, keep_a = centers[pr[0]], centers[pa[0]]
    r = o.energy_forces(pos, sp, off, s.box, aev_table=at, mlp_table=mt,
                        pairs=((pr[0][keep_r], pr[1][keep_r]), (pa[0][keep_a], pa[1][keep_a])))
    return r.F[kl], set(cl[pr[1][pr[0] == kl]].tolist())


def neighborhood_aev(s, at, k):
    """Atom k's symmetry-function row from the oracle on the atoms within
    R_c + 0.5 A of k (the row depends only on k's neighbors within R_c)."""
    rc = at.rc_rad
    box = np.asarray(s.box, np.float64)
    d = s.pos.astype(np.float64) - s.pos[k].astype(np.float64)
    d -= box * np.rint(d / box)
    cl = np.nonzero((d * d).sum(1) < (rc + 0.5) ** 2)[0]
    kl = int(np.nonzero(cl == k)[0][0])
    pos, sp = s.pos[cl], s.species[cl]
    off = np.array([0, cl.size], np.int32)
    pr = pair_list(pos, off, s.box, rc)
    pa = pair_list(pos, off, s.box, at.rc_ang)
    kr, ka = pr[0] == kl, pa[0] == kl
    G, _ = o.aev(pos, sp, off, s.box, at, (pr[0][kr], pr[1][kr]), (pa[0][ka], pa[1][ka]))
    return G[kl]
