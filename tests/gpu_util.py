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


# Force bars of the parity tests (derived in the design notes):
#   FP32 path: relative RMS <= 1e-5 (the contract figure), and no atom's
#     error above 1e-4 of the reference's RMS atomic force (FP32 sums of a few
#     hundred terms err by ~1e-6 of the force scale);
#   BF16 path: relative RMS <= 1e-2, force RMSE <= 1e-2 eV/A, and no atom's
#     error above 5e-2 of the RMS atomic force (BF16 operands round by up to
#     2^-9; an atom's force mixes a few dozen such dE/dG entries).
FORCE_BARS = {"fp32": {"rel": 1e-5, "atom": 1e-4, "rmse": None},
              "bf16": {"rel": 1e-2, "atom": 5e-2, "rmse": 1e-2}}


def check_forces(F, Fref, prec, label=""):
    """Asserts the force bars of `prec`; returns (rel-RMS, worst atom, RMSE)."""
    F = np.asarray(F, np.float64).reshape(-1, 3)
    Fr = np.asarray(Fref, np.float64).reshape(-1, 3)
    if Fr.shape[0] == 0:
        return 0.0, 0.0, 0.0
    d = F - Fr
    rel = float(np.linalg.norm(d) / max(np.linalg.norm(Fr), 1e-300))
    rms_atom = float(np.sqrt(np.mean(np.sum(Fr * Fr, 1))))
    worst = float(np.sqrt(np.sum(d * d, 1)).max() / max(rms_atom, 1e-300))
    rmse = float(np.sqrt(np.mean(d * d)))
    print(f"{label} {prec}: force rel-RMS {rel:.3e}  worst atom {worst:.3e} of RMS|F|="
          f"{rms_atom:.3e}  RMSE {rmse:.3e} eV/A", flush=True)
    b = FORCE_BARS[prec]
    assert np.all(np.isfinite(F))
    assert rel <= b["rel"], rel
    assert worst <= b["atom"], worst
    if b["rmse"] is not None:
        assert rmse <= b["rmse"], rmse
    return rel, worst, rmse
