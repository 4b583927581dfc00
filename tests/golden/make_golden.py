"""Writes the stored oracle values of the test suite.  Calls only ``oracle``
and the ``workloads`` input generators.

* c0_oracle.json: the FP64 oracle's energy and forces for the 24-atom
  four-species molecule (geometry seed 0, weights seed 100).  Guards the
  oracle against unintended changes; not a pin of the method (the paper
  prints no energies or forces).
* water7667_oracle.npz: the oracle on the whole 23,001-atom water box
  (7,667 waters, 61.2 A, seven-element potential, geometry seed 4, weights
  seed 101): total energy E (float64), atomic network outputs E_atom
  (float64 [N], no self energies), forces F (float64 rounded to float32
  [N, 3]; a relative change of at most 6e-8, far below the parity bars), and
  per atom the radial and angular neighbor counts and an order-free checksum
  of the radial neighbor set (the sum over neighbors j of mix32(j), modulo
  2^32, mix32 below).  The whole box takes the oracle about two minutes, too
  long for a test run beside the GPU.

Run: python tests/golden/make_golden.py [c0] [water7667]
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import workloads as w  # noqa: E402


def mix32(j):
    """A 32-bit integer mix of neighbor indices (multiply-xorshift), uint64
    arithmetic masked to 32 bits."""
    x = np.asarray(j, np.uint64) & np.uint64(0xFFFFFFFF)
    x = (x * np.uint64(0x9E3779B1)) & np.uint64(0xFFFFFFFF)
    x ^= x >> np.uint64(15)
    x = (x * np.uint64(0x85EBCA77)) & np.uint64(0xFFFFFFFF)
    x ^= x >> np.uint64(13)
    return x


def neighbor_checksums(I, J, n):
    """Per centre atom: the sum of mix32(j) over its neighbors, modulo 2^32."""
    acc = np.zeros(n, np.uint64)
    np.add.at(acc, np.asarray(I, np.int64), mix32(J))
    return (acc & np.uint64(0xFFFFFFFF)).astype(np.uint32)


def c0():
    s = w.config_system(0)
    r = oracle.energy_forces(s, aev_table=w.aev_table(4), mlp_table=w.mlp_table(4))
    out = {
        "what": "FP64 oracle energy (eV) and forces (eV/A), 24-atom molecule, 4 species",
        "E": [float(x) for x in r.E],
        "F": np.asarray(r.F).tolist(),
        "G_row0_nonzero": {str(int(k)): float(r.G[0, k]) for k in np.nonzero(r.G[0])[0]},
    }
    with open(os.path.join(HERE, "c0_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)


def water7667():
    s = w.config_system(4)
    at, mt = w.aev_table(7), w.mlp_table(7)
    n = s.n_atoms
    Ir, Jr = oracle.pair_list(s.pos, s.mol_offsets, s.box, at.rc_rad)
    Ia, _ = oracle.pair_list(s.pos, s.mol_offsets, s.box, at.rc_ang)
    r = oracle.energy_forces(s, aev_table=at, mlp_table=mt)
    np.savez_compressed(
        os.path.join(HERE, "water7667_oracle.npz"),
        E=np.float64(r.E[0]), E_atom=np.asarray(r.E_atom, np.float64),
        F=np.asarray(r.F, np.float32),
        n_radial=np.bincount(Ir, minlength=n).astype(np.int16),
        n_angular=np.bincount(Ia, minlength=n).astype(np.int16),
        radial_checksum=neighbor_checksums(Ir, Jr, n))


if __name__ == "__main__":
    which = sys.argv[1:] or ["c0", "water7667"]
    for name in which:
        {"c0": c0, "water7667": water7667}[name]()
