"""Atomic environment vectors and their adjoint, float64 (oracle; test use only).

The paper names "the atom-centered symmetry functions used in the ANI family
of potentials" as the operation its optimized kernels compute (Methods,
"Optimization Through NNPOps") and benchmarks ANI-2x (Results, "Performance of
MLPs", Table 3), but prints no formula.  This module writes out the published
ANI (modified Behler-Parrinello) definition:

  f_C(d; R) = 0.5 cos(pi d / R) + 0.5 for d < R, else 0.

  Radial, for each neighbor j of i (float32 predicate at R_cr), m = 0..n_R-1:
    G_i[s_j*n_R + m] += c_R exp(-eta_R (d_ij - R_m)^2) f_C(d_ij; R_cr)

  Angular, for each unordered pair {j, k} of angular neighbors of i
  (predicate at R_ca), a = 0..n_A-1, z = 0..n_Z-1:
    theta = arccos(kappa * cos(angle j-i-k))
    G_i[S*n_R + P(s_j,s_k)*n_A*n_Z + a*n_Z + z] +=
        2^(1-zeta) (1 + cos(theta - theta_z))^zeta
        * exp(-eta_A ((d_ij + d_ik)/2 - R_a)^2) * f_C(d_ij; R_ca) f_C(d_ik; R_ca)

  P(p, q), p <= q, is the upper-triangular index p*S - p(p-1)/2 + (q - p).

c_R (``radial_prefactor``) and kappa (``angle_cos_scale``) are parameters; the
ANI-2x convention is 0.25 and 0.95.  Displacements use the minimum image when
a box is given.  The angle uses ``arccos`` directly.
"""
from __future__ import annotations

import numpy as np

from .neighbors import pair_list


def n_features(S: int, n_r: int, n_a: int, n_z: int) -> int:
    return S * n_r + (S * (S + 1) // 2) * n_a * n_z


def pair_block_index(p, q, S: int):
    lo = np.minimum(p, q)
    hi = np.maximum(p, q)
    return lo * S - (lo * (lo - 1)) // 2 + (hi - lo)


def cutoff(d, R):
    return np.where(d < R, 0.5 * np.cos(np.pi * d / R) + 0.5, 0.0)


def cutoff_grad(d, R):
    return np.where(d < R, -0.5 * (np.pi / R) * np.sin(np.pi * d / R), 0.0)


def displacement(pos64, i, j, box):
    """v_ij = r_j - r_i in float64, minimum image when a box is given (edge
    lengths, or the rows of a reduced triclinic cell: image removed along c,
    b, a in turn)."""
    v = pos64[j] - pos64[i]
    if box is not None:
        B = np.asarray(box, dtype=np.float64)
        if B.shape == (3, 3):
            for k in (2, 1, 0):
                v = v - np.rint(v[:, k] / B[k, k])[:, None] * B[k]
        else:
            v = v - B * np.rint(v / B)
    return v


def _triples(I, J, n_atoms):
    """All unordered pairs {j, k} (j listed before k) of neighbors of each i,
    from a neighbor list sorted by i then j."""
    counts = np.bincount(I, minlength=n_atoms)
    starts = np.concatenate([[0], np.cumsum(counts)])
    TI, TJ, TK = [], [], []
    for c in np.unique(counts):
        if c < 2:
            continue
        atoms = np.nonzero(counts == c)[0]
        a, b = np.triu_indices(c, 1)
        s = starts[atoms][:, None]
        TI.append(np.repeat(atoms, a.size))
        TJ.append((s + a[None, :]).ravel())
        TK.append((s + b[None, :]).ravel())
    if not TI:
        z = np.zeros(0, np.int64)
        return z, z, z
    # TJ/TK index into the pair arrays (positions in the list), not atoms.
    return np.concatenate(TI), np.concatenate(TJ), np.concatenate(TK)


class AEVCache:
    """Geometry and per-term factors kept for the adjoint."""


def aev(pos32, species, mol_offsets, box, t, pairs_r=None, pairs_a=None):
    """G [N, F] float64 and a cache for ``aev_backward``.

    ``pos32`` holds the float32 input positions; float64 positions are also
    accepted (finite-difference checks), in which case the neighbor sets come
    from their float32 rounding unless ``pairs_r``/``pairs_a`` are given."""
    pos = np.asarray(pos32)
    if pos.dtype != np.float64:
        pos = pos.astype(np.float32).astype(np.float64)
    pos32 = pos.astype(np.float32)
    sp = np.asarray(species, dtype=np.int64)
    N = pos.shape[0]
    S, nR, nA, nZ = t.n_species, t.n_r, t.n_a, t.n_z
    F = n_features(S, nR, nA, nZ)
    Rcr = float(t.rc_rad)
    Rca = float(t.rc_ang)
    etaR = float(t.eta_r)
    etaA = float(t.eta_a)
    zeta = float(t.zeta)
    cR = float(t.radial_prefactor)
    kappa = float(t.angle_cos_scale)
    shfR = t.shf_r.astype(np.float64)
    shfA = t.shf_a.astype(np.float64)
    shfZ = t.shf_z.astype(np.float64)

    if pairs_r is None:
        pairs_r = pair_list(pos32, mol_offsets, box, t.rc_rad)
    if pairs_a is None:
        pairs_a = pair_list(pos32, mol_offsets, box, t.rc_ang)
    I, J = pairs_r
    G = np.zeros((N, F))

    # radial terms
    v = displacement(pos, I, J, box)
    d = np.sqrt((v * v).sum(1))
    fc = cutoff(d, Rcr)
    gauss = np.exp(-etaR * (d[:, None] - shfR[None, :]) ** 2)       # [P, nR]
    rad = cR * gauss * fc[:, None]
    cols = sp[J][:, None] * nR + np.arange(nR)[None, :]
    np.add.at(G, (np.repeat(I, nR), cols.ravel()), rad.ravel())

    # angular terms
    IA, JA = pairs_a
    va = displacement(pos, IA, JA, box)
    da = np.sqrt((va * va).sum(1))
    TI, TJ, TK = _triples(IA, JA, N)
    vj, vk = va[TJ], va[TK]
    dj, dk = da[TJ], da[TK]
    cosang = (vj * vk).sum(1) / (dj * dk)
    theta = np.arccos(kappa * cosang)
    base = 1.0 + np.cos(theta[:, None] - shfZ[None, :])               # [T, nZ]
    f1 = 2.0 ** (1.0 - zeta) * base ** zeta
    dbar = 0.5 * (dj + dk)
    f2 = np.exp(-etaA * (dbar[:, None] - shfA[None, :]) ** 2)         # [T, nA]
    fcj = cutoff(dj, Rca)
    fck = cutoff(dk, Rca)
    ang = f2[:, :, None] * f1[:, None, :] * (fcj * fck)[:, None, None]  # [T, nA, nZ]
    blk = pair_block_index(sp[JA[TJ]], sp[JA[TK]], S)
    col0 = S * nR + blk * (nA * nZ)
    cols = col0[:, None] + np.arange(nA * nZ)[None, :]
    np.add.at(G, (np.repeat(TI, nA * nZ), cols.ravel()), ang.reshape(-1))

    c = AEVCache()
    c.__dict__.update(dict(N=N, S=S, nR=nR, nA=nA, nZ=nZ, F=F, I=I, J=J, v=v, d=d,
                           fc=fc, gauss=gauss, IA=IA, JA=JA, TI=TI, TJ=TJ, TK=TK,
                           vj=vj, vk=vk, dj=dj, dk=dk, cosang=cosang, theta=theta,
                           base=base, f1=f1, f2=f2, dbar=dbar, fcj=fcj, fck=fck,
                           col0=col0, cols_r=cols, sp=sp, Rcr=Rcr, Rca=Rca,
                           etaR=etaR, etaA=etaA, zeta=zeta, cR=cR, kappa=kappa,
                           shfR=shfR, shfA=shfA, shfZ=shfZ))
    c.cols_r = sp[J][:, None] * nR + np.arange(nR)[None, :]
    return G, c


def aev_backward(g, c):
    """dE/dr [N, 3] (float64) given g = dE/dG [N, F], by the chain rule."""
    g = np.asarray(g, dtype=np.float64)
    dEdr = np.zeros((c.N, 3))

    # radial: d/dd [c_R exp(-eta (d-R_m)^2) f_C(d)]
    gr = g[c.I[:, None], c.cols_r]                                     # [P, nR]
    fcp = cutoff_grad(c.d, c.Rcr)
    dterm = c.cR * c.gauss * (-2.0 * c.etaR * (c.d[:, None] - c.shfR[None, :])
                              * c.fc[:, None] + fcp[:, None])
    dEdd = (gr * dterm).sum(1)
    u = c.v / c.d[:, None]
    np.add.at(dEdr, c.J, dEdd[:, None] * u)
    np.add.at(dEdr, c.I, -dEdd[:, None] * u)

    if c.TI.size:
        nAZ = c.nA * c.nZ
        ga = g[c.TI[:, None], c.col0[:, None] + np.arange(nAZ)[None, :]]
        ga = ga.reshape(-1, c.nA, c.nZ)
        zeta, kappa = c.zeta, c.kappa
        # d f1 / d theta and d theta / d cos
        df1 = (2.0 ** (1.0 - zeta) * zeta * c.base ** (zeta - 1.0)
               * -np.sin(c.theta[:, None] - c.shfZ[None, :]))        # [T, nZ]
        dtheta = -kappa / np.sqrt(1.0 - (kappa * c.cosang) ** 2)     # [T]
        df2 = c.f2 * (-c.etaA * (c.dbar[:, None] - c.shfA[None, :]))  # d f2 / d d_j
        fcjp = cutoff_grad(c.dj, c.Rca)
        fckp = cutoff_grad(c.dk, c.Rca)
        fcc = c.fcj * c.fck
        dE_dcos = (ga * c.f2[:, :, None] * df1[:, None, :]).sum((1, 2)) * dtheta * fcc
        S0 = (ga * c.f2[:, :, None] * c.f1[:, None, :]).sum((1, 2))
        S1 = (ga * df2[:, :, None] * c.f1[:, None, :]).sum((1, 2))
        dE_ddj = S1 * fcc + S0 * fcjp * c.fck
        dE_ddk = S1 * fcc + S0 * c.fcj * fckp
        dj, dk = c.dj[:, None], c.dk[:, None]
        cs = c.cosang[:, None]
        dcos_dvj = c.vk / (dj * dk) - cs * c.vj / (dj * dj)
        dcos_dvk = c.vj / (dj * dk) - cs * c.vk / (dk * dk)
        gvj = dE_dcos[:, None] * dcos_dvj + dE_ddj[:, None] * c.vj / dj
        gvk = dE_dcos[:, None] * dcos_dvk + dE_ddk[:, None] * c.vk / dk
        np.add.at(dEdr, c.JA[c.TJ], gvj)
        np.add.at(dEdr, c.JA[c.TK], gvk)
        np.add.at(dEdr, c.TI, -(gvj + gvk))
    return dEdr
