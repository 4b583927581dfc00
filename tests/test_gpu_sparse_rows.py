"""Sparse feature rows on the whole-network path.

With forces, one network and BF16 operands, the symmetry-function forward
stores only the k-steps (32 feature columns) that hold a block each atom
touches, and the network kernel runs layer 1 and dE/dG over its tile's
union of those k-steps.  nnp_backward with weight gradients stores whole
rows (the weight gradients read them) and runs the same network kernel: a
skipped k-step adds exact zeros, so in the deterministic mode the two give
the same energies and the same forces bit for bit (dL/dpos = -F for L = the
sum of the energies).  Odd and even element counts cover the rows with and
without the zero gap before the angular blocks.
"""
import numpy as np
import pytest
import torch

import workloads as w
from gpu_util import potential, to_dev

pytestmark = pytest.mark.gpu


def announce(msg):
    print(f"\n[case] {msg}", flush=True)


CASES = {
    "batch64x64-7el": lambda: (w.conformer_batch(64, 64, seed=1), 7),
    "water-box-7el": lambda: (w.water_box(300, 20.8, seed=5, n_species=7), 7),
    "batch32x64-8el": lambda: (w.conformer_batch(32, 64, seed=2, n_species=8), 8),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_sparse_rows_equal_whole_rows(name):
    s, S = CASES[name]()
    announce(f"sparse vs whole feature rows {name} N={s.n_atoms}")
    pot, _, _ = potential(S, "bf16", deterministic=True)
    pos, sp, off = to_dev(s)
    E, F = pot.energy_forces(pos, sp, off, s.box)
    pot.check()
    ones = torch.ones(s.n_mol, dtype=torch.float64, device="cuda")
    g, gw, E2 = pot.backward(pos, sp, off, ones, box=s.box, want_params=True)
    pot.check()
    assert torch.equal(E, E2)
    assert torch.equal(g, -F)
    assert bool(torch.isfinite(gw).all())
    # and a second call on the same workspace after the whole-row one
    E3, F3 = pot.energy_forces(pos, sp, off, s.box)
    pot.check()
    assert torch.equal(E3, E) and torch.equal(F3, F)
