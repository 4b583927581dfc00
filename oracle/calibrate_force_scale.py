"""Recompute the output-layer scale of the synthetic potentials (a script).

Prints RMS |F| (eV/A) of the four-species potential on the 1,500-water box and
of the seven-species potential on the 7,667-water box, both at unit output
scale; the stored scale in ``workloads.params.FORCE_SCALE`` is the rounded
inverse, so that forces are about 1 eV/A.  Run: python -m oracle.calibrate_force_scale
"""
import numpy as np

import workloads as w
from .potential import energy_forces


def main():
    for k, S in ((2, 4), (4, 7)):
        s = w.config_system(k)
        r = energy_forces(s, aev_table=w.aev_table(S), mlp_table=w.mlp_table(S, out_scale=1.0))
        rms = float(np.sqrt((r.F ** 2).sum(1).mean()))
        print(f"config {k}: S={S} RMS|F| at unit scale = {rms:.4f} eV/A -> scale {1.0 / rms:.2f}")


if __name__ == "__main__":
    main()
