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


def _check_against_oracle(pot, at, mt, s, prec, label):
    import oracle as o
    from gpu_util import check_forces
    pos, sp, off = to_dev(s)
    E, F = pot.energy_forces(pos, sp, off, s.box)
    pot.check()
    r = o.energy_forces(s, aev_table=at, mlp_table=mt)
    check_forces(F.cpu().numpy(), r.F, prec, label)
    # a molecule's energy error against the sum of its atomic energies, or
    # the mean atomic energy when that is larger: a one-atom molecule's
    # energy can be a small difference of its network's terms, and its BF16
    # error is then that of one network evaluation (up to 2e-2 of it here)
    mean_atom = np.abs(r.E_atom).mean()
    scale = np.array([max(np.abs(r.E_atom[s.mol_offsets[m]:s.mol_offsets[m + 1]]).sum(),
                          mean_atom) for m in range(s.n_mol)])
    de = np.abs(E.cpu().numpy() - r.E) / scale
    print(f"{label} {prec}: max |dE| / scale {de.max():.3e}")
    assert de.max() <= (1e-5 if prec == "fp32" else 1e-2), de.max()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("S", [1, 3])
def test_few_elements(S, prec):
    # one element (feature rows of 48 columns, 64 with the gap: the layer
    # kernels) and three (240 columns, 256 with the gap: the whole-network
    # kernel on the BF16 path), against the oracle
    mols = []
    for n in (5, 17, 33, 64, 90):
        m = w.single_molecule(n, seed=20 + n, n_species=4)
        sp = np.random.default_rng(60 + n).integers(0, S, n).astype(np.int32)
        mols.append(w.System(m.pos, sp, m.mol_offsets, None, S, f"mol{n}"))
    s = w.pack_molecules(mols, S)
    announce(f"{S} element(s) {prec} N={s.n_atoms}")
    pot, at, mt = potential(S, prec)
    _check_against_oracle(pot, at, mt, s, prec, f"S={S}")


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_isolated_atoms_have_empty_rows(prec):
    # one-atom molecules have no neighbors: their rows touch no k-step, and
    # tiles made only of them run no k-step at all; beside them two-atom and
    # larger molecules of seven elements
    mols = [w.single_molecule(1, seed=40 + k, n_species=7) for k in range(300)]
    mols += [w.single_molecule(2, seed=400 + k, n_species=7) for k in range(40)]
    mols += [w.single_molecule(24, seed=500 + k, n_species=7) for k in range(6)]
    s = w.pack_molecules(mols, 7)
    announce(f"isolated atoms {prec} N={s.n_atoms}")
    pot, at, mt = potential(7, prec)
    _check_against_oracle(pot, at, mt, s, prec, "isolated")
