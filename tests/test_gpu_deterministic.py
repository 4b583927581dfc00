"""Deterministic gather mode (nnp_set_deterministic): forces formed by a
gather over per-entry adjoint rows instead of floating-point atomics.

Every energy and force is then a function of its molecule alone, so a
molecule evaluated alone, at another position of another batch, or in a
second run gives the same bits; and the values still meet the oracle's bars.
"""
import numpy as np
import pytest
import torch

import oracle as o
import workloads as w
from gpu_util import potential, to_dev, check_forces

pytestmark = pytest.mark.gpu


def announce(msg):
    print(f"\n[case] {msg}", flush=True)


_POT = {}


def det_pot(S, prec):
    if (S, prec) not in _POT:
        _POT[(S, prec)] = potential(S, prec, deterministic=True)
    return _POT[(S, prec)]


def _eval(pot, s):
    pos, sp, off = to_dev(s)
    box = None if s.box is None else s.box
    E, F = pot.energy_forces(pos, sp, off, box)
    pot.check()
    return E.cpu().numpy(), F.cpu().numpy()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_alone_equals_mix_bitwise(prec):
    # three molecules of a 64-atom batch, each alone and at other positions
    # of a reordered batch of mixed sizes: the same energy and force bits
    s = w.conformer_batch(24, 64, seed=1)
    serving = w.config_system(3, n_req=12)
    announce(f"deterministic alone vs mix {prec}")
    pot, at, mt = det_pot(7, prec)
    E, F = _eval(pot, s)
    for m in (0, 9, 23):
        a, b = s.mol_offsets[m], s.mol_offsets[m + 1]
        E1, F1 = _eval(pot, s.molecule(m))
        assert E1[0] == E[m], (m, E1[0], E[m])
        assert np.array_equal(F1, F[a:b]), m
        # the molecule between serving-sized molecules, in a second batch
        mols = [serving.molecule(k) for k in range(4)] + [s.molecule(m)] + \
               [serving.molecule(k) for k in range(4, 9)]
        mix = w.pack_molecules(mols, 7)
        E2, F2 = _eval(pot, mix)
        a2, b2 = mix.mol_offsets[4], mix.mol_offsets[5]
        assert E2[4] == E[m], m
        assert np.array_equal(F2[a2:b2], F[a:b]), m
    # and the serving molecules between themselves: alone == in the mix
    Es, Fs = _eval(pot, serving)
    for k in (0, 5, 11):
        a, b = serving.mol_offsets[k], serving.mol_offsets[k + 1]
        E1, F1 = _eval(pot, serving.molecule(k))
        assert E1[0] == Es[k] and np.array_equal(F1, Fs[a:b]), k


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("name", ["c0-mol24", "c1-batch16x64", "box-60w-smallcell",
                                  "c2-water1500"])
def test_gather_forces_match_oracle(name, prec):
    s, S = {"c0-mol24": lambda: (w.config_system(0), 4),
            "c1-batch16x64": lambda: (w.conformer_batch(16, 64, seed=1), 7),
            "box-60w-smallcell": lambda: (w.water_box(60, 12.0, seed=7), 4),
            "c2-water1500": lambda: (w.config_system(2), 4)}[name]()
    announce(f"deterministic vs oracle {name} {prec} N={s.n_atoms}")
    pot, at, mt = det_pot(S, prec)
    E, F = _eval(pot, s)
    r = o.energy_forces(s, aev_table=at, mlp_table=mt)
    check_forces(F, r.F, prec, name)
    scale = np.array([np.abs(r.E_atom[s.mol_offsets[m]:s.mol_offsets[m + 1]]).sum()
                      for m in range(s.n_mol)])
    de = np.abs(E - r.E) / np.maximum(scale, 1e-30)
    assert de.max() <= (1e-5 if prec == "fp32" else 1e-2), de.max()


def test_gather_equals_scatter_and_repeats_on_a_box():
    # the 1,500-water box: the gather's forces agree with the atomic scatter's
    # to rounding, a second run repeats them bit for bit, and the adjoint of
    # L = sum E (nnp_backward, dL/dpos) is exactly their negative
    s = w.config_system(2)
    announce(f"deterministic box repeat N={s.n_atoms}")
    det, _, _ = det_pot(4, "fp32")
    ref, _, _ = potential(4, "fp32")
    E, F = _eval(det, s)
    E2, F2 = _eval(det, s)
    assert np.array_equal(E, E2) and np.array_equal(F, F2)
    Ea, Fa = _eval(ref, s)
    d = np.linalg.norm(F - Fa) / np.linalg.norm(Fa)
    print(f"gather vs scatter rel-RMS {d:.3e}")
    assert d <= 1e-6
    assert abs(E[0] - Ea[0]) <= 1e-9 * np.abs(Ea[0]) + 1e-9
    pos, sp, off = to_dev(s)
    dLdE = torch.ones(1, dtype=torch.float64, device="cuda")
    g, _, _ = det.backward(pos, sp, off, dLdE, box=s.box, want_params=False)
    det.check()
    g = g.cpu().numpy()
    assert np.array_equal(g, -F)


def test_gather_subset_adds_to_caller_rows():
    # subset evaluation adds the forces to the caller's rows in gather mode too
    lig = w.single_molecule(53, seed=3, n_species=7)
    rng = np.random.default_rng(9)
    n_total = 4000
    full = rng.uniform(-30.0, 40.0, size=(n_total, 3)).astype(np.float32)
    idx = rng.choice(n_total, size=53, replace=False).astype(np.int32)
    full[idx] = lig.pos
    F_mm = rng.normal(size=(n_total, 3)).astype(np.float32)
    announce(f"deterministic subset 53 of {n_total}")
    pot, at, mt = det_pot(7, "fp32")
    F_all = torch.from_numpy(F_mm.copy()).cuda()
    pot.energy_forces_subset(torch.from_numpy(idx).cuda(), torch.from_numpy(full).cuda(),
                             torch.from_numpy(lig.species).cuda(),
                             torch.from_numpy(lig.mol_offsets).cuda(), F_all=F_all)
    pot.check()
    F = F_all.cpu().numpy()
    rest = np.setdiff1d(np.arange(n_total), idx)
    assert np.array_equal(F[rest], F_mm[rest])
    _, F_alone = _eval(pot, lig)
    assert np.array_equal(F[idx] - F_mm[idx], (F_alone + F_mm[idx]) - F_mm[idx])
    r = o.energy_forces(lig, aev_table=at, mlp_table=mt)
    check_forces(F[idx] - F_mm[idx], r.F, "fp32", "subset")
