"""Writes tests/golden/c0_oracle.json: the FP64 oracle's energy and forces for
the 24-atom four-species molecule (geometry seed 0, weights seed 100).

Calls only ``oracle`` and the ``workloads`` input generators.  The stored
values guard the oracle against unintended changes; they are not a pin of
the method (the paper prints no energies or forces).
Run: python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import workloads as w  # noqa: E402


def main():
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


if __name__ == "__main__":
    main()
