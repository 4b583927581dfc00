"""GPU parity of the HIP path against the FP64 oracle (through the C ABI).

Bars (written here, derived in the design notes):
* neighbor sets: bit-exact (float32 predicate on both sides);
* symmetry functions: relative RMS <= 2e-6 (FP32 arithmetic against FP64);
* FP32 path: forces relative RMS <= 1e-5, |dE_m| <= 1e-5 * sum_i |E_i|;
* BF16 path: forces relative RMS <= 1e-2, energies relative to sum |E_i| <= 1e-2;
* parameter gradients (FP32 path): relative error <= 1e-4 per layer block.
"""
import os

import numpy as np
import pytest
import torch

import oracle as o
import workloads as w
from oracle.neighbors import pair_list
from gpu_util import potential, to_dev, rel_rms, pair_set_from_ell, check_forces
from neighborhood import neighborhood_reference, neighborhood_aev

pytestmark = pytest.mark.gpu


def announce(msg):
    print(f"\n[case] {msg}", flush=True)


def small_systems():
    return {
        "c0-mol24": (w.config_system(0), 4),
        "c1-batch32x64": (w.conformer_batch(32, 64, seed=1), 7),
        "c3-serving32": (w.config_system(3, n_req=32), 7),
        "box-60w-smallcell": (w.water_box(60, 12.0, seed=7), 4),
        "c2-water1500": (w.config_system(2), 4),
    }


_SYS = {}
_POT = {}


def get_sys(name):
    if not _SYS:
        _SYS.update(small_systems())
    return _SYS[name]


def get_pot(S, prec):
    key = (S, prec)
    if key not in _POT:
        _POT[key] = potential(S, prec)
    return _POT[key]


NAMES = ["c0-mol24", "c1-batch32x64", "c3-serving32", "box-60w-smallcell", "c2-water1500"]


@pytest.mark.parametrize("name", NAMES)
def test_pairs_bit_exact(name):
    s, S = get_sys(name)
    announce(f"pairs {name} N={s.n_atoms}")
    pot, at, mt = get_pot(S, "fp32")
    pos, sp, off = to_dev(s)
    pot.energy_forces(pos, sp, off, s.box, forces=False)
    pot.check()
    counts, nbr = pot.debug_neighbors(s.n_atoms)
    torch.cuda.synchronize()
    I, J = pair_set_from_ell(counts, nbr)
    Io, Jo = pair_list(s.pos, s.mol_offsets, s.box, at.rc_rad)
    assert np.array_equal(I, Io) and np.array_equal(J, Jo)
    # angular neighbors are the first counts[:,1] entries of each row
    c = counts.cpu().numpy()
    nb = nbr.cpu().numpy()
    IA = np.concatenate([np.full(c[i, 1], i) for i in range(s.n_atoms)])
    JA = np.concatenate([nb[i, :c[i, 1]] for i in range(s.n_atoms)])
    o_ = np.lexsort((JA, IA))
    Ia, Ja = pair_list(s.pos, s.mol_offsets, s.box, at.rc_ang)
    assert np.array_equal(IA[o_], Ia) and np.array_equal(JA[o_], Ja)


@pytest.mark.parametrize("name", NAMES)
def test_aev_parity(name):
    s, S = get_sys(name)
    announce(f"aev {name}")
    pot, at, mt = get_pot(S, "fp32")
    pos, sp, off = to_dev(s)
    G = pot.debug_aev(pos, sp, off, s.box).cpu().numpy()
    pot.check()
    Go, _ = o.aev(s.pos, s.species, s.mol_offsets, s.box, at)
    assert G.shape == Go.shape
    err = rel_rms(G, Go)
    print(f"aev rel-RMS {err:.3e}  max|d| {np.abs(G - Go).max():.3e}")
    assert err <= 2e-6
    # exact zeros where the oracle has no contribution
    assert np.all(G[Go == 0] == 0)


def _check_ef(name, prec, f_tol, e_tol):
    s, S = get_sys(name)
    announce(f"energy+forces {name} {prec}")
    pot, at, mt = get_pot(S, prec)
    pos, sp, off = to_dev(s)
    E, F = pot.energy_forces(pos, sp, off, s.box)
    pot.check()
    E = E.cpu().numpy()
    F = F.cpu().numpy()
    r = o.energy_forces(s, aev_table=at, mlp_table=mt)
    scale = np.array([np.abs(r.E_atom[s.mol_offsets[m]:s.mol_offsets[m + 1]]).sum()
                      for m in range(s.n_mol)])
    de = np.abs(E - r.E) / np.maximum(scale, 1e-30)
    print(f"{prec}: max |dE|/sum|E_i| {de.max():.3e}")
    assert de.max() <= e_tol
    check_forces(F, r.F, prec, name)


@pytest.mark.parametrize("name", NAMES)
def test_energy_forces_fp32(name):
    _check_ef(name, "fp32", 1e-5, 1e-5)


@pytest.mark.parametrize("name", NAMES)
def test_energy_forces_bf16(name):
    _check_ef(name, "bf16", 1e-2, 1e-2)


@pytest.mark.parametrize("prec,f_tol,e_tol", [("fp32", 1e-5, 1e-5), ("bf16", 1e-2, 1e-2)])
def test_energy_forces_five_elements(prec, f_tol, e_tol):
    """Five elements (560 features, 576 padded) and hidden widths 224/160/96:
    the first layer's K is not a multiple of the 128-column A chunk, widths
    that are not multiples of 64 take the 32-row wave layout, and no fused
    middle kernel exists for these widths."""
    base = w.conformer_batch(24, 40, seed=3)
    sp = np.random.default_rng(11).integers(0, 5, base.n_atoms).astype(np.int32)
    s = w.System(base.pos, sp, base.mol_offsets, None, 5, "five-elements")
    at = w.aev_table(5)
    mt = w.mlp_table(5, widths=(560, 224, 160, 96, 1))
    announce(f"five elements {prec} N={s.n_atoms}")
    pot, _, _ = potential(5, prec, aev=at, mlp=mt)
    pos, spd, off = to_dev(s)
    E, F = pot.energy_forces(pos, spd, off, None)
    pot.check()
    E = E.cpu().numpy()
    F = F.cpu().numpy()
    r = o.energy_forces(s, aev_table=at, mlp_table=mt)
    scale = np.array([np.abs(r.E_atom[s.mol_offsets[m]:s.mol_offsets[m + 1]]).sum()
                      for m in range(s.n_mol)])
    de = np.abs(E - r.E) / np.maximum(scale, 1e-30)
    print(f"{prec}: max |dE|/sum|E_i| {de.max():.3e}")
    assert de.max() <= e_tol
    check_forces(F, r.F, prec)


def _eight_element_system():
    base = w.conformer_batch(24, 48, seed=8)
    sp = np.random.default_rng(12).integers(0, 8, base.n_atoms).astype(np.int32)
    return w.System(base.pos, sp, base.mol_offsets, None, 8, "eight-elements")


def test_eight_elements_pairs_and_aev():
    """Eight elements: 36 angular pair blocks (F = 1280), so the forward pass
    needs a third 16-block one-hot tile.  Every block is populated."""
    s = _eight_element_system()
    at = w.aev_table(8)
    mt = w.mlp_table(8, widths=(1280, 256, 192, 160, 1))
    announce(f"eight elements pairs + aev N={s.n_atoms}")
    pot, _, _ = potential(8, "fp32", aev=at, mlp=mt)
    pos, spd, off = to_dev(s)
    pot.energy_forces(pos, spd, off, None, forces=False)
    pot.check()
    counts, nbr = pot.debug_neighbors(s.n_atoms)
    I, J = pair_set_from_ell(counts, nbr)
    Io, Jo = pair_list(s.pos, s.mol_offsets, None, at.rc_rad)
    assert np.array_equal(I, Io) and np.array_equal(J, Jo)
    G = pot.debug_aev(pos, spd, off, None).cpu().numpy()
    pot.check()
    Go, _ = o.aev(s.pos, s.species, s.mol_offsets, None, at)
    assert G.shape == Go.shape == (s.n_atoms, 1280)
    # the last four pair blocks (32..35) are populated in this input
    ang0 = 8 * 16
    assert np.abs(Go[:, ang0 + 32 * 32:]).sum(1).astype(bool).sum() > 20
    err = rel_rms(G, Go)
    err_tail = rel_rms(G[:, ang0 + 32 * 32:], Go[:, ang0 + 32 * 32:])
    print(f"aev rel-RMS {err:.3e}, blocks 32-35 {err_tail:.3e}")
    assert err <= 2e-6 and err_tail <= 2e-6
    assert np.all(G[Go == 0] == 0)


@pytest.mark.parametrize("prec,f_tol,e_tol", [("fp32", 1e-5, 1e-5), ("bf16", 1e-2, 1e-2)])
def test_energy_forces_eight_elements(prec, f_tol, e_tol):
    s = _eight_element_system()
    at = w.aev_table(8)
    mt = w.mlp_table(8, widths=(1280, 256, 192, 160, 1))
    announce(f"eight elements {prec} N={s.n_atoms}")
    pot, _, _ = potential(8, prec, aev=at, mlp=mt)
    pos, spd, off = to_dev(s)
    E, F = pot.energy_forces(pos, spd, off, None)
    pot.check()
    E = E.cpu().numpy()
    F = F.cpu().numpy()
    r = o.energy_forces(s, aev_table=at, mlp_table=mt)
    scale = np.array([np.abs(r.E_atom[s.mol_offsets[m]:s.mol_offsets[m + 1]]).sum()
                      for m in range(s.n_mol)])
    de = np.abs(E - r.E) / np.maximum(scale, 1e-30)
    print(f"{prec}: max |dE|/sum|E_i| {de.max():.3e}")
    assert de.max() <= e_tol
    check_forces(F, r.F, prec)


def test_full_batch_512x64():
    s = w.config_system(1)
    announce(f"full batch 512x64 N={s.n_atoms}")
    for prec, ftol, etol in (("fp32", 1e-5, 1e-5), ("bf16", 1e-2, 1e-2)):
        pot, at, mt = get_pot(7, prec)
        pos, sp, off = to_dev(s)
        E, F = pot.energy_forces(pos, sp, off, None)
        pot.check()
        if prec == "fp32":
            counts, nbr = pot.debug_neighbors(s.n_atoms)
            I, J = pair_set_from_ell(counts, nbr)
            Io, Jo = pair_list(s.pos, s.mol_offsets, None, at.rc_rad)
            assert np.array_equal(I, Io) and np.array_equal(J, Jo)
        r = o.energy_forces(s, aev_table=at, mlp_table=mt)
        E = E.cpu().numpy()
        F = F.cpu().numpy()
        scale = np.abs(r.E_atom).reshape(512, 64).sum(1)
        print(f"{prec}: max dE rel {np.max(np.abs(E - r.E) / scale):.3e}")
        assert np.max(np.abs(E - r.E) / scale) <= etol
        check_forces(F, r.F, prec, "512x64")


def test_full_batch_512x64_bench_capacity():
    """The full batch at the neighbor capacity the benchmark times (64: the
    molecule adjoint then runs 16 waves per workgroup), both precisions."""
    s = w.config_system(1)
    announce(f"full batch 512x64 at capacity 64 N={s.n_atoms}")
    r = None
    for prec, ftol, etol in (("fp32", 1e-5, 1e-5), ("bf16", 1e-2, 1e-2)):
        pot, at, mt = potential(7, prec, max_neighbors=64)
        pos, sp, off = to_dev(s)
        E, F = pot.energy_forces(pos, sp, off, None)
        pot.check()
        if r is None:
            r = o.energy_forces(s, aev_table=at, mlp_table=mt)
        E = E.cpu().numpy()
        F = F.cpu().numpy()
        scale = np.abs(r.E_atom).reshape(512, 64).sum(1)
        print(f"{prec}: max dE rel {np.max(np.abs(E - r.E) / scale):.3e}")
        assert np.max(np.abs(E - r.E) / scale) <= etol
        check_forces(F, r.F, prec, "512x64")


def test_water7667_sampled():
    """The 23,001-atom water box in the benchmark's configuration (neighbor
    capacity 128), both precisions: neighbor lists and forces of 12 sampled
    atoms against the oracle on each atom's neighborhood (the whole box is
    too large for the oracle in a test)."""
    s = w.config_system(4)
    announce(f"water box 7667 sampled N={s.n_atoms}")
    at, mt = w.aev_table(7), w.mlp_table(7)
    ks = np.random.default_rng(5).choice(s.n_atoms, 12, replace=False)
    ref = {int(k): neighborhood_reference(s, at, mt, int(k)) for k in ks}
    for prec, ftol in (("fp32", 1e-5), ("bf16", 1e-2)):
        pot, _, _ = potential(7, prec)
        pos, sp, off = to_dev(s)
        E, F = pot.energy_forces(pos, sp, off, s.box)
        pot.check()
        F = F.cpu().numpy()
        if prec == "fp32":
            counts, nbr = pot.debug_neighbors(s.n_atoms)
            c, nb = counts.cpu().numpy(), nbr.cpu().numpy()
            for k, (_, nset) in ref.items():
                assert set(nb[k, :c[k, 0]].tolist()) == nset, k
        Fg = np.stack([F[k] for k in ref])
        Fr = np.stack([v[0] for v in ref.values()])
        print(f"{prec}: sampled force rel-RMS {rel_rms(Fg, Fr):.3e}")
        assert rel_rms(Fg, Fr) <= ftol


def _mix32(j):
    """The 32-bit mix of neighbor indices that tests/golden/make_golden.py
    sums into its per-atom radial-set checksums (multiply-xorshift)."""
    x = np.asarray(j, np.uint64) & np.uint64(0xFFFFFFFF)
    x = (x * np.uint64(0x9E3779B1)) & np.uint64(0xFFFFFFFF)
    x ^= x >> np.uint64(15)
    x = (x * np.uint64(0x85EBCA77)) & np.uint64(0xFFFFFFFF)
    x ^= x >> np.uint64(13)
    return x


# Atomic energies E_i (network outputs) against the oracle, per atom:
# |dE_i| <= bar * mean_j |E_j|.  FP32: 1e-5 (the energy bar of the molecules,
# applied atom by atom); BF16: 2e-2 (operands rounded to 8-bit mantissas, a
# per-atom error of a few 2^-9 of the size of the terms).
ATOM_E_BARS = {"fp32": 1e-5, "bf16": 2e-2}


def test_water7667_whole_box():
    """The 23,001-atom water box in the benchmark's configuration (neighbor
    capacity 128), both precisions, against the oracle on the whole box
    (tests/golden/water7667_oracle.npz, written by make_golden.py, which
    calls only the oracle): every atom's radial and angular neighbor counts
    and radial-set checksum (bit-exact), the total energy, every atomic
    energy and every force; and 160 sampled symmetry-function rows against
    the oracle on each atom's neighborhood."""
    s = w.config_system(4)
    announce(f"water box 7667 whole box N={s.n_atoms}")
    g = np.load(os.path.join(os.path.dirname(__file__), "golden", "water7667_oracle.npz"))
    Ea_o, F_o, E_o = g["E_atom"], g["F"].astype(np.float64), float(g["E"])
    assert Ea_o.shape == (s.n_atoms,)
    at = w.aev_table(7)
    pos, sp, off = to_dev(s)
    for prec in ("fp32", "bf16"):
        pot, _, _ = potential(7, prec)
        E, F = pot.energy_forces(pos, sp, off, s.box)
        pot.check()
        Ea = pot.debug_atom_energies(s.n_atoms, 1, s.box)[0].cpu().numpy().astype(np.float64)
        if prec == "fp32":
            counts, nbr = pot.debug_neighbors(s.n_atoms)
            c, nb = counts.cpu().numpy(), nbr.cpu().numpy().astype(np.int64)
            assert np.array_equal(c[:, 0], g["n_radial"])
            assert np.array_equal(c[:, 1], g["n_angular"])
            cap = nb.shape[1]
            valid = np.arange(cap)[None, :] < c[:, :1]
            mixed = np.where(valid, _mix32(np.where(valid, nb, 0)), np.uint64(0))
            cks = (mixed.sum(1, dtype=np.uint64) & np.uint64(0xFFFFFFFF)).astype(np.uint32)
            assert np.array_equal(cks, g["radial_checksum"])
        scale = np.abs(Ea_o).sum()
        dE = abs(E.item() - E_o) / scale
        de_atom = np.abs(Ea - Ea_o).max() / np.abs(Ea_o).mean()
        print(f"{prec}: |dE|/sum|E_i| {dE:.3e}  worst |dE_i|/mean|E_i| {de_atom:.3e}")
        assert dE <= (1e-5 if prec == "fp32" else 1e-2)
        assert de_atom <= ATOM_E_BARS[prec]
        check_forces(F.cpu().numpy(), F_o, prec, "water7667")
    ks = np.random.default_rng(6).choice(s.n_atoms, 160, replace=False)
    pot, _, _ = potential(7, "fp32")
    G = pot.debug_aev(pos, sp, off, s.box)
    pot.check()
    Gk = G[torch.from_numpy(ks).cuda()].cpu().numpy()
    Go = np.stack([neighborhood_aev(s, at, int(k)) for k in ks])
    err = rel_rms(Gk, Go)
    print(f"sampled AEV rows rel-RMS {err:.3e}")
    assert err <= 2e-6
    assert np.all(Gk[Go == 0] == 0)


def _many_small(n_mol, seed):
    """n_mol molecules of 0..6 atoms (about one in seven empty), 7 elements."""
    rng = np.random.default_rng(seed)
    mols = []
    for m in range(n_mol):
        n = int(rng.integers(0, 7))
        if n == 0:
            mols.append(w.System(np.zeros((0, 3), np.float32), np.zeros(0, np.int32),
                                 np.array([0, 0], np.int32), None, 7))
        else:
            mols.append(w.single_molecule(n, seed=1000 + m, n_species=7))
    return w.pack_molecules(mols, 7, f"many-small-{n_mol}")


def _check_against_oracle(s, S, prec, f_tol, e_tol, pairs=False):
    """Energies against a per-molecule scale: sum_i |E_i|, but for BF16 at
    least n_m times the mean |E_i| of the whole input.  BF16 rounds the
    activations and weights, so its error per atom follows the typical size
    of the terms, not E_i itself, which for a one- or two-atom molecule can
    nearly cancel."""
    pot, at, mt = get_pot(S, prec)
    pos, sp, off = to_dev(s)
    E, F = pot.energy_forces(pos, sp, off, None)
    pot.check()
    if pairs:
        counts, nbr = pot.debug_neighbors(s.n_atoms)
        I, J = pair_set_from_ell(counts, nbr)
        Io, Jo = pair_list(s.pos, s.mol_offsets, None, at.rc_rad)
        assert np.array_equal(I, Io) and np.array_equal(J, Jo)
    r = o.energy_forces(s, aev_table=at, mlp_table=mt)
    E = E.cpu().numpy()
    F = F.cpu().numpy()
    scale = np.array([np.abs(r.E_atom[s.mol_offsets[m]:s.mol_offsets[m + 1]]).sum()
                      for m in range(s.n_mol)])
    if prec == "bf16":
        scale = np.maximum(scale, np.diff(s.mol_offsets) * np.abs(r.E_atom).mean())
    empty = np.diff(s.mol_offsets) == 0
    assert np.all(E[empty] == r.E[empty])  # both 0: no atoms, no self energies
    de = np.abs(E - r.E)[~empty] / np.maximum(scale[~empty], 1e-30)
    print(f"{prec}: max |dE|/sum|E_i| {de.max():.3e}")
    assert de.max() <= e_tol
    check_forces(F, r.F, prec)


@pytest.mark.parametrize("prec,f_tol,e_tol", [("fp32", 1e-5, 1e-5), ("bf16", 1e-2, 1e-2)])
def test_many_small_molecules(prec, f_tol, e_tol):
    """2,500 molecules (more than the 1,024 offsets each staging block samples,
    so the molecule search ends with global loads), empty ones among them."""
    s = _many_small(2500, seed=11)
    announce(f"many small molecules {prec} n_mol={s.n_mol} N={s.n_atoms}")
    _check_against_oracle(s, 7, prec, f_tol, e_tol, pairs=prec == "fp32")


def test_molecule_batch_above_fused_sort_limit():
    """1,040 x 64 atoms = 66,560 > 65,536: the species sort takes the
    scan-kernel path and the pair scan its own launch."""
    s = w.conformer_batch(1040, 64, seed=1)
    announce(f"molecule batch above the fused-sort limit N={s.n_atoms}")
    _check_against_oracle(s, 7, "fp32", 1e-5, 1e-5, pairs=True)


def test_batch_position_independence():
    # a molecule alone and inside a batch: same pairs, same energy bits, forces
    # equal up to the order of atomic additions
    s = w.conformer_batch(16, 64, seed=1)
    announce("alone vs in batch")
    pot, at, mt = get_pot(7, "fp32")
    pos, sp, off = to_dev(s)
    E, F = pot.energy_forces(pos, sp, off, None)
    m = 9
    one = s.molecule(m)
    p1, s1, o1 = to_dev(one)
    E1, F1 = pot.energy_forces(p1, s1, o1, None)
    pot.check()
    E = E.cpu().numpy()
    F = F.cpu().numpy()
    assert E1.cpu().numpy()[0] == E[m]
    a, b = s.mol_offsets[m], s.mol_offsets[m + 1]
    assert rel_rms(F1.cpu().numpy(), F[a:b]) <= 1e-6


def test_parameter_gradients_fp32():
    s = w.conformer_batch(8, 64, seed=1)
    announce("parameter gradients fp32")
    pot, at, mt = get_pot(7, "fp32")
    pos, sp, off = to_dev(s)
    rng = np.random.default_rng(4)
    dLdE = rng.normal(size=s.n_mol)
    gp, gw, E = pot.backward(pos, sp, off, torch.from_numpy(dLdE).cuda())
    pot.check()
    gw_o, dpos_o = o.weight_gradients(s, aev_table=at, mlp_table=mt, dL_dE=dLdE)
    gw = gw.cpu().numpy()
    print(f"dL/dparams rel-RMS {rel_rms(gw, gw_o):.3e}; dL/dpos rel-RMS "
          f"{rel_rms(gp.cpu().numpy(), dpos_o):.3e}")
    # per (species, layer) block
    o_ = 0
    present = set(int(x) for x in s.species)
    for sp_ in range(7):
        for l in range(4):
            n = mt.W[sp_][l].size + mt.b[sp_][l].size
            blk = slice(o_, o_ + n)
            if sp_ in present:
                assert rel_rms(gw[blk], gw_o[blk]) <= 1e-4, (sp_, l)
            else:
                assert np.all(gw[blk] == 0)
            o_ += n
    assert rel_rms(gp.cpu().numpy(), dpos_o) <= 1e-5


@pytest.mark.parametrize("S", [7, 4])
def test_parameter_gradients_bf16(S):
    # BF16 network operands (activations, deltas and weights rounded to
    # 8-bit mantissas, FP32 accumulation): each operand carries a relative
    # rounding error up to 2^-9, so the per-block gradients are held to 3e-2
    # relative RMS and dL/dpos to 1e-2, the force bar of the BF16 path.
    s = w.conformer_batch(8, 64, seed=1) if S == 7 else w.water_box(60, 12.0, seed=7)
    announce(f"parameter gradients bf16, {S} elements, {s.n_atoms} atoms")
    pot, at, mt = get_pot(S, "bf16")
    pos, sp, off = to_dev(s)
    rng = np.random.default_rng(5)
    dLdE = rng.normal(size=s.n_mol)
    gp, gw, E = pot.backward(pos, sp, off, torch.from_numpy(dLdE).cuda(), box=s.box)
    pot.check()
    gw_o, dpos_o = o.weight_gradients(s, aev_table=at, mlp_table=mt, dL_dE=dLdE)
    gw = gw.cpu().numpy()
    worst = 0.0
    o_ = 0
    present = set(int(x) for x in s.species)
    for sp_ in range(S):
        for l in range(4):
            n = mt.W[sp_][l].size + mt.b[sp_][l].size
            blk = slice(o_, o_ + n)
            if sp_ in present:
                err = rel_rms(gw[blk], gw_o[blk])
                worst = max(worst, err)
                assert err <= 3e-2, (sp_, l, err)
            else:
                assert np.all(gw[blk] == 0)
            o_ += n
    dp = rel_rms(gp.cpu().numpy(), dpos_o)
    print(f"worst block dL/dparams rel-RMS {worst:.3e}; dL/dpos rel-RMS {dp:.3e}")
    assert dp <= 1e-2


@pytest.mark.parametrize("prec,blk_tol,pos_tol", [("fp32", 1e-4, 1e-5), ("bf16", 3e-2, 1e-2)])
def test_parameter_gradients_full_batch(prec, blk_tol, pos_tol):
    """Weight gradients of the full 512 x 64 batch (32,768 atoms, seven
    elements) through nnp_backward, per (element, layer) block against the
    oracle, with the same bars as the small cases."""
    s = w.config_system(1)
    announce(f"parameter gradients full batch {prec} N={s.n_atoms}")
    pot, at, mt = get_pot(7, prec)
    pos, sp, off = to_dev(s)
    dLdE = np.random.default_rng(8).normal(size=s.n_mol)
    gp, gw, E = pot.backward(pos, sp, off, torch.from_numpy(dLdE).cuda())
    pot.check()
    gw_o, dpos_o = o.weight_gradients(s, aev_table=at, mlp_table=mt, dL_dE=dLdE)
    gw = gw.cpu().numpy()
    worst = 0.0
    o_ = 0
    present = set(int(x) for x in s.species)
    for sp_ in range(7):
        for l in range(4):
            n = mt.W[sp_][l].size + mt.b[sp_][l].size
            blk = slice(o_, o_ + n)
            if sp_ in present:
                err = rel_rms(gw[blk], gw_o[blk])
                worst = max(worst, err)
                assert err <= blk_tol, (sp_, l, err)
            else:
                assert np.all(gw[blk] == 0)
            o_ += n
    dp = rel_rms(gp.cpu().numpy(), dpos_o)
    print(f"{prec}: worst block dL/dparams rel-RMS {worst:.3e}; dL/dpos rel-RMS {dp:.3e}")
    assert dp <= pos_tol


def test_autograd_function_matches_forces():
    from paper_2310_03121_amd import NNPFunction
    s = w.config_system(0)
    announce("autograd function")
    pot, at, mt = get_pot(4, "fp32")
    pos, sp, off = to_dev(s)
    params = torch.from_numpy(mt.flat()).cuda().requires_grad_(True)
    x = pos.clone().requires_grad_(True)
    E = NNPFunction.apply(x, params, pot, sp, off, None)
    E.sum().backward()
    r = o.energy_forces(s, aev_table=at, mlp_table=mt)
    assert rel_rms(-x.grad.cpu().numpy(), r.F) <= 1e-5
    gw_o, _ = o.weight_gradients(s, aev_table=at, mlp_table=mt)
    assert rel_rms(params.grad.cpu().numpy(), gw_o) <= 1e-4


def test_fp32_finite_difference_gradcheck():
    s = w.config_system(0)
    announce("fp32 finite differences on the GPU")
    pot, at, mt = get_pot(4, "fp32")
    pos, sp, off = to_dev(s)
    E0, F = pot.energy_forces(pos, sp, off, None)
    F = F.cpu().numpy()
    h = 2e-3
    rng = np.random.default_rng(0)
    errs = []
    for i in rng.choice(s.n_atoms, 6, replace=False):
        for c in range(3):
            xp = pos.clone(); xp[i, c] += h
            xm = pos.clone(); xm[i, c] -= h
            ep, _ = pot.energy_forces(xp, sp, off, None, forces=False)
            em, _ = pot.energy_forces(xm, sp, off, None, forces=False)
            dx = float(xp[i, c] - xm[i, c])
            fd = -(ep.item() - em.item()) / dx
            errs.append((fd, F[i, c]))
    a = np.array(errs)
    assert rel_rms(a[:, 0], a[:, 1]) <= 2e-2


def test_water7667_weight_gradient_finite_differences():
    """Weight gradients of the whole 23,001-atom water box (FP32 path,
    nnp_backward) against central differences of the GPU energy: for each
    element present (H, O) and each layer, the weight with the largest
    gradient.  Bar 2e-3 relative: the energy is an FP64 sum of FP32 atomic
    energies, so a difference of two evaluations carries ~1e-5 eV of rounding
    noise, against g h of about 1e-2 eV or more here."""
    s = w.config_system(4)
    announce(f"weight-gradient finite differences, water box N={s.n_atoms}")
    pot, at, mt = potential(7, "fp32")
    pos, sp, off = to_dev(s)
    dLdE = torch.ones(1, dtype=torch.float64, device="cuda")
    _, gw, E0 = pot.backward(pos, sp, off, dLdE, box=s.box, want_pos=False)
    pot.check()
    gw = gw.cpu().numpy().astype(np.float64)
    flat = mt.flat().astype(np.float32)
    picks = []
    o_ = 0
    for sp_ in range(7):
        for l in range(4):
            nW, nb = mt.W[sp_][l].size, mt.b[sp_][l].size
            if sp_ in (0, 3):
                picks.append(o_ + int(np.argmax(np.abs(gw[o_:o_ + nW]))))
            o_ += nW + nb
    worst = 0.0
    for idx in picks:
        h = np.float32(1e-3)
        pp, pm = flat.copy(), flat.copy()
        pp[idx] += h
        pm[idx] -= h
        pot.set_params(torch.from_numpy(pp).cuda())
        ep, _ = pot.energy_forces(pos, sp, off, s.box, forces=False)
        pot.set_params(torch.from_numpy(pm).cuda())
        em, _ = pot.energy_forces(pos, sp, off, s.box, forces=False)
        pot.check()
        fd = (ep.item() - em.item()) / (float(pp[idx]) - float(pm[idx]))
        err = abs(fd - gw[idx]) / abs(gw[idx])
        worst = max(worst, err)
        print(f"param {idx}: backward {gw[idx]:.6e}  central difference {fd:.6e}  rel {err:.2e}")
        assert err <= 2e-3, (idx, gw[idx], fd)
    pot.set_params(torch.from_numpy(flat).cuda())
    print(f"worst relative error {worst:.2e} over {len(picks)} weights")


def test_device_errors_are_reported():
    from paper_2310_03121_amd import NNPError
    announce("device status: species, non-finite, capacity; host: box")
    pot, at, mt = get_pot(4, "fp32")
    s = w.config_system(0)
    pos, sp, off = to_dev(s)
    bad = sp.clone(); bad[3] = 9
    pot.energy_forces(pos, bad, off, None)
    with pytest.raises(NNPError) as e:
        pot.check()
    assert e.value.code == 2
    nanpos = pos.clone(); nanpos[5, 1] = float("nan")
    pot.energy_forces(nanpos, sp, off, None)
    with pytest.raises(NNPError) as e:
        pot.check()
    assert e.value.code == 7
    pot.energy_forces(pos, sp, off, None)
    pot.check()  # clean again
    with pytest.raises(NNPError) as e:
        pot.energy_forces(pos, sp, off, (9.0, 20.0, 20.0))
    assert e.value.code == 3
    small, _, _ = potential(4, "fp32", max_neighbors=16)
    wb = w.water_box(60, 12.0, seed=7)
    p2, s2, o2 = to_dev(wb)
    small.energy_forces(p2, s2, o2, wb.box)
    with pytest.raises(NNPError) as e:
        small.check()
    assert e.value.code == 4


def test_empty_and_isolated():
    announce("empty molecules and isolated atoms")
    pot, at, mt = get_pot(4, "fp32")
    s = w.System(np.array([[0, 0, 0], [30, 0, 0], [0, 30, 0]], np.float32),
                 np.array([0, 1, 3], np.int32), np.array([0, 0, 2, 2, 3], np.int32), None, 4)
    pos, sp, off = to_dev(s)
    E, F = pot.energy_forces(pos, sp, off, None)
    pot.check()
    r = o.energy_forces(s, aev_table=at, mlp_table=mt)
    np.testing.assert_allclose(E.cpu().numpy(), r.E, rtol=1e-6, atol=1e-7)
    assert np.all(F.cpu().numpy() == 0)


def test_graph_replay_matches_eager():
    # replays of a captured evaluation, with positions changed in place and
    # eager evaluations and synchronisations between the replays
    s = w.conformer_batch(16, 64, seed=1)
    announce("graph replay vs eager, 16x64 batch, 4 replays")
    for prec in ("fp32", "bf16"):
        pot, at, mt = get_pot(7, prec)
        pos, sp, off = to_dev(s)
        g = pot.capture(pos, sp, off, None)
        rng = torch.Generator(device="cpu").manual_seed(5)
        for k in range(4):
            with torch.no_grad():
                pos.add_((torch.randn(pos.shape, generator=rng) * 0.01).cuda())
            torch.cuda.synchronize()
            E_ref, F_ref = pot.energy_forces(pos, sp, off, None)
            torch.cuda.synchronize()
            g.launch()
            g.synchronize()
            g.check()
            assert torch.equal(g.E.cpu(), E_ref.cpu()), (prec, k)
            assert rel_rms(g.F.cpu().numpy(), F_ref.cpu().numpy()) <= 1e-6, (prec, k)


# ------------------------------------------------------------------ ensembles
def _ensemble_case(S):
    if S == 7:
        s = w.conformer_batch(12, 64, seed=1)
        seeds = (101, 102, 103)
    else:
        s = w.config_system(0)
        seeds = (100, 107, 108)
    return s, w.aev_table(S), [w.mlp_table(S, seed=k) for k in seeds]


@pytest.mark.parametrize("S,prec,f_tol,e_tol", [(7, "fp32", 1e-5, 1e-5), (7, "bf16", 1e-2, 1e-2),
                                                (4, "fp32", 1e-5, 1e-5), (4, "bf16", 1e-2, 1e-2)])
def test_ensemble_energy_forces(S, prec, f_tol, e_tol):
    s, at, members = _ensemble_case(S)
    announce(f"ensemble of {len(members)} S={S} {prec} N={s.n_atoms}")
    from paper_2310_03121_amd import Potential
    pot = Potential.ensemble_from_tables(at, members, precision=prec)
    pos, sp, off = to_dev(s)
    E, F = pot.energy_forces(pos, sp, off, s.box)
    E_only, _ = pot.energy_forces(pos, sp, off, s.box, forces=False)
    pot.check()
    E, F, E_only = E.cpu().numpy(), F.cpu().numpy(), E_only.cpu().numpy()
    r = o.ensemble_energy_forces(s, aev_table=at, mlp_tables=members)
    scale = np.array([np.abs(r.E_atom[s.mol_offsets[m]:s.mol_offsets[m + 1]]).sum()
                      for m in range(s.n_mol)])
    de = np.abs(E - r.E) / np.maximum(scale, 1e-30)
    print(f"ensemble {prec}: max |dE|/sum|E_i| {de.max():.3e}")
    assert de.max() <= e_tol
    check_forces(F, r.F, prec, "ensemble")
    # the energy-only path runs the forward kernels alone; same mean energy
    assert np.abs(E_only - E).max() <= 1e-6 * max(1.0, np.abs(E).max())


def test_ensemble_of_one_equals_single_network():
    s, at, members = _ensemble_case(7)
    announce("ensemble of one vs single network")
    from paper_2310_03121_amd import Potential
    pos, sp, off = to_dev(s)
    for prec in ("fp32", "bf16"):
        a = Potential.from_tables(at, members[0], precision=prec)
        b = Potential.ensemble_from_tables(at, members[:1], precision=prec)
        Ea, Fa = a.energy_forces(pos, sp, off, None)
        Eb, Fb = b.energy_forces(pos, sp, off, None)
        a.check()
        b.check()
        # energies are reduced in a fixed order (bitwise equal); forces are
        # scattered with atomics, whose order varies from run to run
        assert torch.equal(Ea, Eb)
        assert rel_rms(Fb.cpu().numpy(), Fa.cpu().numpy()) <= 1e-6


def test_ensemble_rejects_weight_gradients():
    s, at, members = _ensemble_case(4)
    announce("ensemble weight gradients are rejected")
    from paper_2310_03121_amd import Potential
    from paper_2310_03121_amd.capi import NNPError
    pot = Potential.ensemble_from_tables(at, members, precision="fp32")
    pos, sp, off = to_dev(s)
    dLdE = torch.ones(s.n_mol, dtype=torch.float64, device="cuda")
    with pytest.raises(NNPError):
        pot.backward(pos, sp, off, dLdE, None, want_pos=True, want_params=True)
    gp, gw, _ = pot.backward(pos, sp, off, dLdE, None, want_pos=True, want_params=False)
    assert gw is None and torch.isfinite(gp).all()


# ------------------------------------------------ subset of a larger system
@pytest.mark.parametrize("prec,f_tol,e_tol", [("fp32", 1e-5, 1e-5), ("bf16", 1e-2, 1e-2)])
def test_subset_in_larger_system(prec, f_tol, e_tol):
    # a 53-atom, seven-element ligand scattered through a 6,000-atom system
    # whose other rows already hold (random) classical forces
    lig = w.single_molecule(53, seed=3, n_species=7)
    rng = np.random.default_rng(9)
    n_total = 6000
    full = rng.uniform(-30.0, 40.0, size=(n_total, 3)).astype(np.float32)
    idx = rng.choice(n_total, size=53, replace=False).astype(np.int32)
    full[idx] = lig.pos
    F_mm = rng.normal(size=(n_total, 3)).astype(np.float32)
    announce(f"subset {prec}: 53 of {n_total} atoms")
    pot, at, mt = get_pot(7, prec)
    sp = torch.from_numpy(lig.species).cuda()
    off = torch.from_numpy(lig.mol_offsets).cuda()
    F_all = torch.from_numpy(F_mm.copy()).cuda()
    E = pot.energy_forces_subset(torch.from_numpy(idx).cuda(), torch.from_numpy(full).cuda(), sp,
                                 off, F_all=F_all)
    pot.check()
    Eo, Fo = o.subset_energy_forces(full, idx, lig.species, lig.mol_offsets, None, aev_table=at,
                                    mlp_table=mt, F_other=F_mm)
    r = o.energy_forces(lig, aev_table=at, mlp_table=mt)
    F = F_all.cpu().numpy()
    rest = np.setdiff1d(np.arange(n_total), idx)
    assert np.array_equal(F[rest], F_mm[rest])  # untouched
    de = abs(E.item() - Eo[0]) / np.abs(r.E_atom).sum()
    print(f"subset {prec}: |dE|/sum|E_i| {de:.3e}")
    assert de <= e_tol
    check_forces(F[idx] - F_mm[idx], Fo[idx] - F_mm[idx], prec, "subset")


def test_subset_rejects_rows_outside_the_system():
    lig = w.single_molecule(24, seed=3, n_species=4)
    announce("subset with an out-of-range row")
    pot, at, mt = get_pot(4, "fp32")
    n_total = 100
    full = torch.zeros((n_total, 3), dtype=torch.float32, device="cuda")
    idx = torch.arange(24, dtype=torch.int32, device="cuda")
    idx[5] = n_total + 7
    F_all = torch.zeros((n_total, 3), dtype=torch.float32, device="cuda")
    from paper_2310_03121_amd.capi import NNPError
    pot.energy_forces_subset(idx, full, torch.from_numpy(lig.species).cuda(),
                             torch.from_numpy(lig.mol_offsets).cuda(), F_all=F_all)
    with pytest.raises(NNPError):
        pot.check()


# ------------------------------------------------------------ triclinic box
_TRIC = np.array([[24.0, 0.0, 0.0], [5.0, 22.0, 0.0], [-6.0, 7.0, 21.0]], dtype=np.float32)


def _tric_pot(S, prec):
    key = ("tric", S, prec)
    if key not in _POT:
        _POT[key] = potential(S, prec, triclinic=True)
    return _POT[key]


def test_triclinic_pairs_aev_and_forces():
    s = w.triclinic_system(800, _TRIC, seed=5)
    announce(f"triclinic box, {s.n_atoms} atoms")
    pot, at, mt = _tric_pot(4, "fp32")
    pos, sp, off = to_dev(s)
    pot.energy_forces(pos, sp, off, s.box, forces=False)
    pot.check()
    counts, nbr = pot.debug_neighbors(s.n_atoms)
    I, J = pair_set_from_ell(counts, nbr)
    Io, Jo = pair_list(s.pos, s.mol_offsets, s.box, at.rc_rad)
    assert np.array_equal(I, Io) and np.array_equal(J, Jo)
    G = pot.debug_aev(pos, sp, off, s.box).cpu().numpy()
    Go, _ = o.aev(s.pos, s.species, s.mol_offsets, s.box, at)
    assert rel_rms(G, Go) <= 2e-6
    r = o.energy_forces(s, aev_table=at, mlp_table=mt)
    for prec, f_tol, e_tol in (("fp32", 1e-5, 1e-5), ("bf16", 1e-2, 1e-2)):
        p, _, _ = _tric_pot(4, prec)
        E, F = p.energy_forces(pos, sp, off, s.box)
        p.check()
        de = abs(E.item() - r.E[0]) / np.abs(r.E_atom).sum()
        print(f"triclinic {prec}: |dE|/sum|E_i| {de:.3e}")
        assert de <= e_tol
        check_forces(F.cpu().numpy(), r.F, prec, "triclinic")


def test_triclinic_without_tilt_equals_orthorhombic():
    s, S = get_sys("c2-water1500")
    announce("zero-tilt triclinic cell vs orthorhombic box")
    ortho, at, mt = get_pot(S, "fp32")
    tric, _, _ = _tric_pot(S, "fp32")
    pos, sp, off = to_dev(s)
    E0, F0 = ortho.energy_forces(pos, sp, off, s.box)
    E1, F1 = tric.energy_forces(pos, sp, off, np.diag(np.asarray(s.box, np.float32)))
    ortho.check()
    tric.check()
    assert torch.equal(E0, E1)
    assert rel_rms(F1.cpu().numpy(), F0.cpu().numpy()) <= 1e-6


def test_triclinic_rejects_unreduced_cells():
    announce("triclinic cell checks")
    s = w.triclinic_system(100, _TRIC, seed=6)
    pot, at, mt = _tric_pot(4, "fp32")
    pos, sp, off = to_dev(s)
    from paper_2310_03121_amd.capi import NNPError
    bad = _TRIC.copy()
    bad[1, 0] = 13.0  # |bx| > ax / 2
    with pytest.raises(NNPError):
        pot.energy_forces(pos, sp, off, bad)
