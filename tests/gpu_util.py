"""Helpers of the GPU tests: build potentials and move seeded systems to the GPU."""
import numpy as np
import torch

import workloads as w


def potential(S, precision="fp32", aev=None, mlp=None, **kw):
    from paper_2310_03121_amd import Potential
    aev = aev or w.aev_table(S)
    mlp = mlp or w.mlp_table(S)
    return Potential.from_tables(aev, mlp, precision=precision, **kw), aev, mlp


def to_dev(s):
    dev = "cuda"
    return (torch.from_numpy(np.ascontiguousarray(s.pos)).to(dev),
            torch.from_numpy(np.ascontiguousarray(s.species)).to(dev),
            torch.from_numpy(np.ascontiguousarray(s.mol_offsets)).to(dev))


def rel_rms(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def pair_set_from_ell(counts, nbr):
    counts = counts.cpu().numpy()
    nbr = nbr.cpu().numpy()
    I, J = [], []
    for i in range(counts.shape[0]):
        k = counts[i, 0]
        I.append(np.full(k, i))
        J.append(nbr[i, :k])
    I = np.concatenate(I) if I else np.zeros(0, np.int64)
    J = np.concatenate(J) if J else np.zeros(0, np.int64)
    o = np.lexsort((J, I))
    return I[o].astype(np.int64), J[o].astype(np.int64)
