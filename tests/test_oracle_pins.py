"""Pins of the FP64 oracle against facts that do not come from the oracle:
hand-derived closed forms, brute force on tiny inputs, symmetry invariants of
the energy, finite differences, and special cases with known answers.

Each closed form below is worked out by hand in its comment; the oracle is
never compared with a retyped copy of its own formula.
"""
import math

import numpy as np
import pytest

import oracle as o
import workloads as w
from oracle.neighbors import pair_list, pair_list_loops

f32 = np.float32


def _sys(pos, species, box=None, S=4):
    pos = np.asarray(pos, dtype=np.float32)
    return w.System(pos, np.asarray(species, np.int32), np.array([0, len(pos)], np.int32),
                    None if box is None else np.asarray(box, np.float32), S)


# ---------------------------------------------------------------- pair sets


def test_pairs_match_bruteforce_loops_no_box():
    rng = np.random.default_rng(11)
    pos = rng.uniform(0, 6, (30, 3)).astype(np.float32)
    off = np.array([0, 13, 30], np.int32)
    for rc in (3.5, 5.1):
        a = pair_list(pos, off, None, rc)
        b = pair_list_loops(pos, off, None, rc)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
        # no cross-molecule pairs
        mol = np.repeat([0, 1], [13, 17])
        assert np.all(mol[a[0]] == mol[a[1]])


def test_pairs_match_bruteforce_loops_box():
    rng = np.random.default_rng(12)
    L = np.array([11.0, 12.5, 10.2], np.float32)
    pos = (rng.uniform(0, 1, (40, 3)) * L).astype(np.float32)
    off = np.array([0, 40], np.int32)
    a = pair_list(pos, off, L, 5.1)
    b = pair_list_loops(pos, off, L, 5.1)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert a[0].size > 0


def test_pair_cutoff_is_strict_in_float32():
    rc = f32(5.1)
    below = np.nextafter(rc, f32(0))
    # d2 = fl32(5.1f * 5.1f) equals rc^2 exactly: excluded (strict <).
    I, _ = pair_list(np.array([[0, 0, 0], [rc, 0, 0]], np.float32), [0, 2], None, 5.1)
    assert I.size == 0
    # one ulp closer: fl32(X*X) rounds below rc^2 (ulp of X^2 ~ 1.9e-6 < 2*5.1*4.8e-7).
    I, J = pair_list(np.array([[0, 0, 0], [below, 0, 0]], np.float32), [0, 2], None, 5.1)
    assert list(zip(I, J)) == [(0, 1), (1, 0)]


def test_pair_minimum_image():
    L = np.array([10.0, 10.0, 10.0], np.float32)
    # 0.5 and 9.5 are 1.0 apart through the face; 9.0 apart directly.
    pos = np.array([[0.5, 5, 5], [9.5, 5, 5]], np.float32)
    I, _ = pair_list(pos, [0, 2], L, 3.5)
    assert I.size == 2
    I, _ = pair_list(pos, [0, 2], None, 3.5)
    assert I.size == 0


# ------------------------------------------------------ closed-form AEV values


def test_radial_dimer_closed_form():
    # eta_R = 0 makes every Gaussian 1, so each radial slot of the partner's
    # species block is c_R * f_C(d).  At d = R/2: f_C = cos(pi/2)/2 + 1/2 = 1/2,
    # so the slot is 0.25 * 0.5 = 0.125.  At d = R/3: f_C = 1/4 + 1/2 = 3/4,
    # slot 0.1875.  At d = 2R/3: f_C = -1/4 + 1/2 = 1/4, slot 0.0625.
    t = w.aev_table(4, eta_r=0.0)
    R = float(t.rc_rad)
    for frac, want in ((0.5, 0.125), (1 / 3, 0.1875), (2 / 3, 0.0625)):
        x = f32(R * frac)
        s = _sys([[0, 0, 0], [x, 0, 0]], [1, 3])
        G, _ = o.aev(s.pos, s.species, s.mol_offsets, None, t)
        # atom 0 (species 1) sees species 3: columns 48..63; atom 1 sees 1: 16..31
        assert np.allclose(G[0, 48:64], want, rtol=1e-6, atol=0)
        assert np.allclose(G[1, 16:32], want, rtol=1e-6, atol=0)
        rest0 = np.delete(G[0], np.arange(48, 64))
        rest1 = np.delete(G[1], np.arange(16, 32))
        assert np.all(rest0 == 0) and np.all(rest1 == 0)
    # Exact-value check at d = R/2 independent of the cosine evaluation:
    s = _sys([[0, 0, 0], [f32(R / 2), 0, 0]], [0, 0])
    G, _ = o.aev(s.pos, s.species, s.mol_offsets, None, t)
    assert abs(G[0, 0] - 0.125) < 1e-12


def test_radial_gaussian_half_width():
    # A shift equal to d gives exp(0) = 1; shifts at d -/+ delta with
    # eta * delta^2 = ln 2 give exp(-ln 2) = 1/2 each.  With d = R/2 the slots
    # are 0.125, 0.0625, 0.0625.
    R = float(f32(5.1))
    d = f32(R / 2)
    delta = 0.25
    t = w.aev_table(4, eta_r=math.log(2) / delta ** 2,
                    shf_r=[float(d) - delta, float(d), float(d) + delta] + [0.0] * 13)
    s = _sys([[0, 0, 0], [d, 0, 0]], [2, 2])
    G, _ = o.aev(s.pos, s.species, s.mol_offsets, None, t)
    np.testing.assert_allclose(G[0, 32:35], [0.0625, 0.125, 0.0625], rtol=2e-6)


def _equilateral(a):
    h = a * math.sqrt(3) / 2
    return [[0, 0, 0], [a, 0, 0], [a / 2, h, 0]]


def test_angular_equilateral_trimer_closed_form():
    # Side a = R_ca/2, so every angular cutoff factor is f_C = 1/2 and the
    # product is 1/4.  Each vertex angle is 60 deg, cos = 1/2, so
    # theta = arccos(0.95 * 0.5) = arccos(0.475).  With angle shift
    # theta_0 = arccos(0.475): 2^(1-zeta) (1 + cos 0)^zeta = 2.  With
    # theta_1 = theta_0 + pi/2 and zeta = 2: 2^(-1) (1 + 0)^2 = 1/2.
    # eta_A = 0 makes the radial factor 1.  Each atom has exactly one
    # unordered neighbor pair, so slot values are 2 * 1/4 = 0.5 (z = 0) and
    # 0.5 * 1/4 = 0.125 (z = 1) for every a.
    # Species (1, 2, 2): atom 0 sees the pair (2, 2) -> block P(2,2) = 7;
    # atoms 1 and 2 see (1, 2) -> block P(1,2) = 5 (upper-triangular order
    # (0,0) (0,1) (0,2) (0,3) (1,1) (1,2) (1,3) (2,2) (2,3) (3,3)).
    th0 = math.acos(0.475)
    t = w.aev_table(4, eta_a=0.0, zeta=2.0,
                    shf_z=[th0, th0 + math.pi / 2, 0, 0, 0, 0, 0, 0])
    a = float(t.rc_ang) / 2
    s = _sys(_equilateral(a), [1, 2, 2])
    G, _ = o.aev(s.pos, s.species, s.mol_offsets, None, t)
    base = 4 * 16
    for atom, blk in ((0, 7), (1, 5), (2, 5)):
        block = G[atom, base + blk * 32: base + (blk + 1) * 32].reshape(4, 8)
        np.testing.assert_allclose(block[:, 0], 0.5, rtol=2e-6)
        np.testing.assert_allclose(block[:, 1], 0.125, rtol=2e-6)
        others = np.delete(G[atom, base:], np.arange(blk * 32, (blk + 1) * 32))
        assert np.all(others == 0)


def test_angular_right_angle_is_independent_of_kappa():
    # cos = 0 at a right angle, so theta = arccos(0) = pi/2 for any kappa; with
    # shift pi/2 and zeta = 1 the angular factor is 2^0 (1 + 1) = 2.  Legs of
    # R_ca/2 give f_C^2 = 1/4, so the slot is 0.5 for kappa = 0.95 and 0.5.
    for kappa in (0.95, 0.5):
        t = w.aev_table(4, eta_a=0.0, zeta=1.0, angle_cos_scale=kappa,
                        shf_z=[math.pi / 2] + [0.0] * 7)
        a = float(t.rc_ang) / 2
        s = _sys([[0, 0, 0], [a, 0, 0], [0, a, 0]], [0, 0, 0])
        G, _ = o.aev(s.pos, s.species, s.mol_offsets, None, t)
        np.testing.assert_allclose(G[0, 64:64 + 32:8], 0.5, rtol=2e-6)


def test_angular_radial_shift_half_width():
    # (d_ij + d_ik)/2 = a for the equilateral trimer.  Shifts a - delta, a,
    # a + delta with eta_A delta^2 = ln 2 give radial factors 1/2, 1, 1/2.
    th0 = math.acos(0.475)
    delta = 0.2
    t0 = w.aev_table(4)
    a = float(t0.rc_ang) / 2
    t = w.aev_table(4, eta_a=math.log(2) / delta ** 2, zeta=2.0,
                    shf_a=[a - delta, a, a + delta, 0.0],
                    shf_z=[th0] + [0.0] * 7)
    s = _sys(_equilateral(a), [0, 0, 0])
    G, _ = o.aev(s.pos, s.species, s.mol_offsets, None, t)
    np.testing.assert_allclose(G[0, 64:64 + 24:8], [0.25, 0.5, 0.25], rtol=2e-6)


def test_pair_block_index_enumeration():
    S = 7
    want = 0
    for p in range(S):
        for q in range(p, S):
            assert o.pair_block_index(p, q, S) == want
            assert o.pair_block_index(q, p, S) == want
            want += 1
    assert want == 28
    assert o.n_features(7, 16, 4, 8) == 1008 and o.n_features(4, 16, 4, 8) == 384


# ------------------------------------------------------------------- networks


def test_celu_special_values():
    a = 0.1
    assert o.celu(0.0, a) == 0.0
    assert o.celu(2.5, a) == 2.5
    # alpha (exp(-ln 2) - 1) = -alpha / 2
    assert abs(o.celu(-a * math.log(2), a) + a / 2) < 1e-15
    assert abs(o.celu(-50.0, a) + a) < 1e-15
    # continuous first derivative at 0; derivative equals 1 + CELU(x)/alpha for x <= 0
    assert o.celu_grad(0.0, a) == 1.0 and o.celu_grad(1e-9, a) == 1.0
    x = np.linspace(-1, 0, 11)
    np.testing.assert_allclose(o.celu_grad(x, a), 1 + o.celu(x, a) / a, rtol=1e-12)


def test_zero_output_layer_gives_bias_energy_and_no_force():
    s = w.config_system(0)
    at = w.aev_table(4)
    mt = w.mlp_table(4)
    for sp in range(4):
        mt.W[sp][-1][:] = 0
        mt.b[sp][-1][:] = np.float32(0.5 + sp)
    r = o.energy_forces(s, aev_table=at, mlp_table=mt)
    want = sum(0.5 + float(f32(0.5 + sp)) - 0.5 for sp in s.species)
    assert abs(r.E[0] - want) < 1e-12
    assert np.all(r.F == 0)


def test_identity_regime_is_affine():
    # Huge positive hidden biases put every CELU on its identity branch, so the
    # atomic energy is an affine function of the AEV row.
    mt = w.mlp_table(4)
    for sp in range(4):
        for l in range(mt.n_layers - 1):
            mt.b[sp][l][:] = 1e4
    rng = np.random.default_rng(5)
    G1 = rng.uniform(0, 1, (6, 384))
    G2 = rng.uniform(0, 1, (6, 384))
    sp = np.array([0, 1, 2, 3, 0, 1])
    e = lambda G: o.mlp_forward(G, sp, mt)[0]
    lhs = e(G1 + G2) - e(G1) - e(G2) + e(np.zeros_like(G1))
    assert np.max(np.abs(lhs)) < 1e-8 * np.max(np.abs(e(G1)))


def test_isolated_atoms():
    # Atoms farther apart than R_cr have zero AEV; E is the sum of each
    # network at zero input; forces vanish.
    at, mt = w.aev_table(4), w.mlp_table(4)
    s = _sys([[0, 0, 0], [20, 0, 0], [0, 20, 0]], [0, 1, 3])
    r = o.energy_forces(s, aev_table=at, mlp_table=mt)
    assert np.all(r.G == 0) and np.all(r.F == 0)
    e0, _ = o.mlp_forward(np.zeros((3, 384)), np.array([0, 1, 3]), mt)
    assert abs(r.E[0] - e0.sum()) < 1e-14


# ----------------------------------------------------------- invariants of E, F


def _tables(S):
    return w.aev_table(S), w.mlp_table(S)


def _fixed_pairs(s, at):
    return (pair_list(s.pos, s.mol_offsets, s.box, at.rc_rad),
            pair_list(s.pos, s.mol_offsets, s.box, at.rc_ang))


def test_rotation_translation_invariance():
    s = w.config_system(0)
    at, mt = _tables(4)
    pairs = _fixed_pairs(s, at)
    x = s.pos.astype(np.float64)
    r0 = o.energy_forces(x, s.species, s.mol_offsets, None, aev_table=at, mlp_table=mt, pairs=pairs)
    th = 0.7
    Rz = np.array([[math.cos(th), -math.sin(th), 0], [math.sin(th), math.cos(th), 0], [0, 0, 1]])
    Rx = np.array([[1, 0, 0], [0, math.cos(1.3), -math.sin(1.3)], [0, math.sin(1.3), math.cos(1.3)]])
    R = Rx @ Rz
    y = x @ R.T + np.array([3.0, -7.0, 1.5])
    r1 = o.energy_forces(y, s.species, s.mol_offsets, None, aev_table=at, mlp_table=mt, pairs=pairs)
    assert abs(r1.E[0] - r0.E[0]) <= 1e-12 * abs(r0.E[0])
    np.testing.assert_allclose(r1.F, r0.F @ R.T, atol=1e-12 * np.abs(r0.F).max())


def test_periodic_translation_invariance():
    s = w.water_box(60, 12.0, seed=7)
    at, mt = _tables(4)
    r0 = o.energy_forces(s, aev_table=at, mlp_table=mt)
    shift = np.array([3.3, -1.2, 7.9])
    x = np.mod(s.pos.astype(np.float64) + shift, 12.0)
    pairs = _fixed_pairs(s, at)
    r1 = o.energy_forces(x, s.species, s.mol_offsets, s.box, aev_table=at, mlp_table=mt,
                         pairs=pairs)
    assert abs(r1.E[0] - r0.E[0]) <= 1e-11 * abs(r0.E[0])
    np.testing.assert_allclose(r1.F, r0.F, atol=1e-10)


def test_same_species_permutation_invariance():
    s = w.config_system(0)
    at, mt = _tables(4)
    r0 = o.energy_forces(s, aev_table=at, mlp_table=mt)
    rng = np.random.default_rng(3)
    perm = np.arange(s.n_atoms)
    for sp in range(4):
        idx = np.nonzero(s.species == sp)[0]
        perm[idx] = rng.permutation(idx)
    s2 = _sys(s.pos[perm], s.species[perm])
    r1 = o.energy_forces(s2, aev_table=at, mlp_table=mt)
    assert abs(r1.E[0] - r0.E[0]) <= 1e-12 * abs(r0.E[0])
    np.testing.assert_allclose(r1.F, r0.F[perm], atol=1e-12)


def test_net_force_and_torque_vanish():
    s = w.config_system(0)
    at, mt = _tables(4)
    r = o.energy_forces(s, aev_table=at, mlp_table=mt)
    scale = np.abs(r.F).max()
    assert np.all(np.abs(r.F.sum(0)) < 1e-12 * scale * s.n_atoms)
    torque = np.cross(s.pos.astype(np.float64), r.F).sum(0)
    assert np.all(np.abs(torque) < 1e-11 * scale * s.n_atoms)
    sb = w.water_box(60, 12.0, seed=7)
    rb = o.energy_forces(sb, aev_table=at, mlp_table=mt)
    assert np.all(np.abs(rb.F.sum(0)) < 1e-11 * np.abs(rb.F).max() * sb.n_atoms)


def _central_diff_forces(s, at, mt, h=1e-5, atoms=None):
    pairs = _fixed_pairs(s, at)
    x = s.pos.astype(np.float64)
    atoms = range(s.n_atoms) if atoms is None else atoms
    out = {}
    for i in atoms:
        for c in range(3):
            xp = x.copy(); xp[i, c] += h
            xm = x.copy(); xm[i, c] -= h
            ep = o.energy(xp, s.species, s.mol_offsets, s.box, at, mt, pairs).sum()
            em = o.energy(xm, s.species, s.mol_offsets, s.box, at, mt, pairs).sum()
            out[(i, c)] = -(ep - em) / (2 * h)
    return out


@pytest.mark.parametrize("which", ["molecule", "water"])
def test_forces_are_central_differences(which):
    if which == "molecule":
        s = w.config_system(0)
        S = 4
        atoms = None
    else:
        s = w.water_box(60, 12.0, seed=7)
        S = 7
        atoms = list(range(0, 180, 7))
    at, mt = _tables(S)
    r = o.energy_forces(s, aev_table=at, mlp_table=mt)
    fd = _central_diff_forces(s, at, mt, atoms=atoms)
    a = np.array([fd[k] for k in fd])
    b = np.array([r.F[k] for k in fd])
    assert np.linalg.norm(a - b) <= 1e-6 * np.linalg.norm(b)


def test_energy_continuous_at_cutoffs():
    # A dimer crossing R_cr and an angular pair crossing R_ca: the jump
    # |E(R - eps) - E(R + eps)| must shrink as eps^2 (f_C and f_C' vanish at R).
    at, mt = _tables(4)
    R = float(at.rc_rad)

    def dimer_E(d):
        s = _sys([[0, 0, 0], [d, 0, 0]], [1, 2])
        return o.energy_forces(s, aev_table=at, mlp_table=mt, forces=False).E[0]

    jumps = []
    for eps in (1e-2, 1e-3):
        jumps.append(abs(dimer_E(R - eps) - dimer_E(R + eps)))
    assert jumps[1] < jumps[0] / 50

    # Angular: the part of E that the triple {j, k} contributes, measured as
    # E with k in i's angular list minus E without it (same positions), must
    # vanish as eps^2 when k sits eps inside R_ca.
    Ra = float(at.rc_ang)

    def triple_part(eps):
        s = _sys([[0, 0, 0], [1.2, 0, 0], [0, Ra - eps, 0]], [0, 1, 2])
        pr = pair_list(s.pos, s.mol_offsets, None, at.rc_rad)
        IA, JA = pair_list(s.pos, s.mol_offsets, None, at.rc_ang)
        keep = ~(((IA == 0) & (JA == 2)) | ((IA == 2) & (JA == 0)))
        e_with = o.energy(s.pos, s.species, s.mol_offsets, None, at, mt, (pr, (IA, JA)))[0]
        e_wo = o.energy(s.pos, s.species, s.mol_offsets, None, at, mt,
                        (pr, (IA[keep], JA[keep])))[0]
        return abs(e_with - e_wo)

    jumps = [triple_part(e) for e in (1e-2, 1e-3)]
    assert jumps[0] > 0 and jumps[1] < jumps[0] / 50


def test_weight_gradients_are_central_differences():
    s = w.single_molecule(12, seed=4, n_species=4)
    at = w.aev_table(4)
    mt = w.mlp_table(4)
    # float64 parameter copies so that small perturbations are exact
    mt64 = mt.from_flat(mt.flat().astype(np.float64))
    grad, _ = o.weight_gradients(s, aev_table=at, mlp_table=mt64)
    theta = mt64.flat().astype(np.float64)
    rng = np.random.default_rng(9)
    present = set(int(x) for x in s.species)
    sizes = [[mt.W[sp][l].size + mt.b[sp][l].size for l in range(mt.n_layers)] for sp in range(4)]
    per_sp = [sum(z) for z in sizes]
    idx = []
    for sp in present:
        base = sum(per_sp[:sp])
        idx.extend(base + rng.choice(per_sp[sp], 12, replace=False))
    h = 1e-6
    for k in idx:
        tp = theta.copy(); tp[k] += h
        tm = theta.copy(); tm[k] -= h
        ep = o.energy(s.pos, s.species, s.mol_offsets, None, at, mt64.from_flat(tp)).sum()
        em = o.energy(s.pos, s.species, s.mol_offsets, None, at, mt64.from_flat(tm)).sum()
        fd = (ep - em) / (2 * h)
        assert abs(fd - grad[k]) <= 1e-6 * max(1.0, abs(grad[k])), (k, fd, grad[k])


# ----------------------------------------------------------------- integrator


def _md_setup():
    s = w.single_molecule(10, seed=21, n_species=4)
    at, mt = _tables(4)
    m = w.MASS_AMU[s.species]
    rng = np.random.default_rng(2)
    v = w.maxwell_boltzmann(s.species, 300.0, rng)

    def ff(x32):
        r = o.energy_forces(x32, s.species, s.mol_offsets, None, aev_table=at, mlp_table=mt)
        return r.E, r.F

    return s, m, v, ff


def test_velocity_verlet_time_reversible():
    s, m, v, ff = _md_setup()
    x0 = s.pos.astype(np.float64)
    x1, v1, _ = o.velocity_verlet(x0, v, m, ff, 0.5, 40)
    x2, v2, _ = o.velocity_verlet(x1, -v1, m, ff, 0.5, 40)
    assert np.max(np.abs(x2 - x0)) < 1e-5
    assert np.max(np.abs(v2 + v)) < 1e-6


def test_velocity_verlet_energy_error_scales_as_dt_squared():
    s, m, v, ff = _md_setup()
    x0 = s.pos.astype(np.float64)
    errs = []
    for dt in (0.4, 0.2):
        n = int(round(20 / dt))
        _, _, rec = o.velocity_verlet(x0, v, m, ff, dt, n)
        e = np.array([r[1] + r[2] for r in rec])
        errs.append(np.max(np.abs(e - e[0])))
    ratio = errs[0] / errs[1]
    assert 2.5 < ratio < 6.0, ratio


def test_kinetic_energy_equipartition_units():
    # <KE> per degree of freedom is k_B T / 2 for Maxwell-Boltzmann draws.
    rng = np.random.default_rng(8)
    sp = rng.integers(0, 7, 20000)
    v = w.maxwell_boltzmann(sp, 300.0, rng)
    ke = o.kinetic_energy(v, w.MASS_AMU[sp])
    kT = 8.617333262e-5 * 300.0
    assert abs(ke / (1.5 * kT * sp.size) - 1) < 0.02


def test_golden_regression_c0():
    import json
    import os
    p = os.path.join(os.path.dirname(__file__), "golden", "c0_oracle.json")
    ref = json.load(open(p))
    s = w.config_system(0)
    r = o.energy_forces(s, aev_table=w.aev_table(4), mlp_table=w.mlp_table(4))
    assert abs(r.E[0] - ref["E"][0]) < 1e-12 * abs(ref["E"][0])
    np.testing.assert_allclose(r.F, np.array(ref["F"]), rtol=0, atol=1e-12)


# ---------------------------------------------------------------- ensembles
def _ens_case():
    s = w.single_molecule(24, seed=0, n_species=4)
    at = w.aev_table(4)
    members = [w.mlp_table(4, seed=100 + k) for k in range(3)]
    return s, at, members


def test_ensemble_of_one_is_the_model():
    s, at, (m0, _, _) = _ens_case()
    a = o.energy_forces(s, aev_table=at, mlp_table=m0)
    b = o.ensemble_energy_forces(s, aev_table=at, mlp_tables=[m0])
    assert np.array_equal(a.E, b.E) and np.array_equal(a.F, b.F)


def test_ensemble_of_identical_copies_is_the_model():
    s, at, (m0, _, _) = _ens_case()
    a = o.energy_forces(s, aev_table=at, mlp_table=m0)
    b = o.ensemble_energy_forces(s, aev_table=at, mlp_tables=[m0, m0, m0])
    np.testing.assert_allclose(b.E, a.E, rtol=1e-14, atol=0)
    np.testing.assert_allclose(b.F, a.F, rtol=1e-13, atol=1e-15)


def test_ensemble_is_the_mean_of_separate_evaluations():
    # each member evaluated on its own (own symmetry functions, own adjoint)
    s, at, members = _ens_case()
    sep = [o.energy_forces(s, aev_table=at, mlp_table=m) for m in members]
    ens = o.ensemble_energy_forces(s, aev_table=at, mlp_tables=members)
    E = sum(r.E for r in sep) / 3
    F = sum(r.F for r in sep) / 3
    np.testing.assert_allclose(ens.E, E, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(ens.F, F, rtol=1e-11, atol=1e-12)
    # and it differs from every member (the members really differ)
    assert all(np.abs(r.E - ens.E).max() > 1e-3 for r in sep)


def test_ensemble_with_negated_twin_cancels_exactly():
    # a member whose output layer is negated gives -E_i exactly: the mean of
    # the pair leaves only the self energies, and no force at all
    s, at, (m0, _, _) = _ens_case()
    se = np.array([-0.6, -38.0, -54.7, -75.2])
    m0 = w.MLPTable(m0.widths, m0.W, m0.b, se, m0.celu_alpha)
    Wn = [[W.copy() for W in ws] for ws in m0.W]
    bn = [[b.copy() for b in bs] for bs in m0.b]
    for sp in range(4):
        Wn[sp][-1] = -Wn[sp][-1]
        bn[sp][-1] = -bn[sp][-1]
    twin = w.MLPTable(m0.widths, Wn, bn, se, m0.celu_alpha)
    r = o.ensemble_energy_forces(s, aev_table=at, mlp_tables=[m0, twin])
    assert np.all(r.E_atom == 0.0) and np.all(r.F == 0.0)
    np.testing.assert_allclose(r.E, [se[s.species].sum()], rtol=1e-15)


# ------------------------------------------------- Langevin (LF-Middle) + RNG
def test_philox_known_answers():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")
    rows = [ln.split() for ln in open(path) if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        assert o.philox4x32_10(v[0:4], v[4:6]) == tuple(v[6:10])


def test_box_muller_normals_are_standard():
    from oracle.rng import normals
    z = np.concatenate([normals(5000, step, seed=12345).ravel() for step in (0, 1)])
    n = z.size
    assert abs(z.mean()) < 5 / math.sqrt(n)
    assert abs(z.var() - 1.0) < 5 * math.sqrt(2.0 / n)
    # distinct steps and atoms draw independent numbers
    a, b = z[: n // 2], z[n // 2:]
    assert abs(np.corrcoef(a, b)[0, 1]) < 5 / math.sqrt(n // 2)
    assert abs(((z ** 4).mean()) - 3.0) < 0.15  # kurtosis of a normal


def _spring(k=0.5):
    def ff(x32):
        x = x32.astype(np.float64)
        return np.array([0.5 * k * np.sum(x * x)]), -k * x
    return ff


def test_langevin_without_friction_is_velocity_verlet():
    # c = 1 removes the noise; leapfrog from v_{-1/2} = v_0 - dt/2 a(x_0)
    # then visits exactly the velocity-Verlet positions
    rng = np.random.default_rng(0)
    x0 = rng.normal(size=(6, 3))
    v0 = rng.normal(scale=0.01, size=(6, 3))
    m = np.array([1.008, 12.011, 15.999, 1.008, 14.007, 32.06])
    ff = _spring()
    dt = 0.5
    _, F0 = ff(x0.astype(np.float32))
    vh = v0 - 0.5 * dt * o.integrator.ACC_UNIT * F0 / m[:, None]
    for n in (1, 7, 25):
        xl, _, _ = o.langevin_middle(x0, vh, m, ff, dt, n, 300.0, 0.0, seed=1)
        xv, _, _ = o.velocity_verlet(x0, v0, m, ff, dt, n)
        np.testing.assert_allclose(xl, xv, rtol=0, atol=1e-12)


def test_langevin_free_particles_follow_ornstein_uhlenbeck():
    # no force: v_{n+1/2} = c v + sqrt(1 - c^2) sigma R is an exact OU
    # process, so from v = 0 the variance after n steps is
    # sigma^2 (1 - c^(2n)), sigma^2 = kB T / m in A^2/fs^2
    N, n, T, gam, dt = 4000, 12, 300.0, 100.0, 0.5
    m = np.full(N, 12.011)
    zero = lambda x32: (np.zeros(1), np.zeros_like(x32, dtype=np.float64))
    _, v, _ = o.langevin_middle(np.zeros((N, 3)), np.zeros((N, 3)), m, zero, dt, n, T, gam,
                                seed=7)
    c = math.exp(-gam * 1e-3 * dt)
    var = o.integrator.KB_EV * T * o.integrator.ACC_UNIT / 12.011 * (1 - c ** (2 * n))
    z = v.ravel()
    assert abs(z.var() / var - 1.0) < 5 * math.sqrt(2.0 / z.size)
    assert abs(z.mean()) < 5 * math.sqrt(var / z.size)


# ------------------------------------------------- subset of a larger system
def _subset_case():
    lig = w.single_molecule(24, seed=3, n_species=4)
    rng = np.random.default_rng(8)
    mm = rng.uniform(-20.0, 30.0, size=(300, 3)).astype(np.float32)
    full = np.concatenate([mm, lig.pos]).astype(np.float32)
    perm = rng.permutation(full.shape[0])
    full = full[perm]
    inv = np.empty_like(perm)
    inv[perm] = np.arange(perm.size)
    idx = inv[300 + np.arange(24)]  # rows of the ligand atoms after the shuffle
    return lig, full, idx


def test_subset_is_the_subset_alone():
    lig, full, idx = _subset_case()
    at, mt = w.aev_table(4), w.mlp_table(4)
    assert np.array_equal(full[idx], lig.pos)
    E, F = o.subset_energy_forces(full, idx, lig.species, lig.mol_offsets, None, aev_table=at,
                                  mlp_table=mt)
    r = o.energy_forces(lig, aev_table=at, mlp_table=mt)
    assert np.array_equal(E, r.E) and np.array_equal(F[idx], r.F)
    rest = np.setdiff1d(np.arange(full.shape[0]), idx)
    assert np.all(F[rest] == 0.0)


def test_subset_ignores_the_other_atoms_and_keeps_their_forces():
    # mechanical embedding: moving atoms outside the subset changes nothing
    # in the subset's energy, and their forces are passed through untouched
    lig, full, idx = _subset_case()
    at, mt = w.aev_table(4), w.mlp_table(4)
    rest = np.setdiff1d(np.arange(full.shape[0]), idx)
    moved = full.copy()
    moved[rest] += np.float32(0.37)
    Fo = np.random.default_rng(2).normal(size=full.shape)
    E1, F1 = o.subset_energy_forces(full, idx, lig.species, lig.mol_offsets, None,
                                    aev_table=at, mlp_table=mt, F_other=Fo)
    E2, F2 = o.subset_energy_forces(moved, idx, lig.species, lig.mol_offsets, None,
                                    aev_table=at, mlp_table=mt, F_other=Fo)
    assert np.array_equal(E1, E2) and np.array_equal(F1, F2)
    assert np.array_equal(F1[rest], Fo[rest])
    # the subset's forces still sum to zero (momentum conservation)
    assert np.abs((F1[idx] - Fo[idx]).sum(0)).max() < 1e-10


# ---------------------------------------------------------- triclinic boxes
_TRIC = np.array([[16.0, 0.0, 0.0], [3.0, 15.0, 0.0], [-4.0, 5.0, 14.0]], dtype=np.float32)


def test_triclinic_without_tilt_is_orthorhombic():
    from oracle.neighbors import pair_list
    s = w.water_box(60, 12.0, seed=7)
    at, mt = w.aev_table(4), w.mlp_table(4)
    L = np.asarray(s.box, dtype=np.float32)
    tri = np.diag(L).astype(np.float32)
    for rc in (at.rc_rad, at.rc_ang):
        a = pair_list(s.pos, s.mol_offsets, L, rc)
        b = pair_list(s.pos, s.mol_offsets, tri, rc)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    ra = o.energy_forces(s.pos, s.species, s.mol_offsets, L, aev_table=at, mlp_table=mt)
    rb = o.energy_forces(s.pos, s.species, s.mol_offsets, tri, aev_table=at, mlp_table=mt)
    assert np.array_equal(ra.E, rb.E) and np.array_equal(ra.F, rb.F)


def test_triclinic_pairs_match_an_image_search():
    # every pair closer than the cutoff in some periodic image, and only
    # those (pairs within 1e-4 A of the cutoff are left out: float32 decides)
    from oracle.neighbors import pair_list
    s = w.triclinic_system(250, _TRIC, seed=2)
    rc = 5.1
    I, J = pair_list(s.pos, s.mol_offsets, _TRIC, rc)
    got = set(zip(I.tolist(), J.tolist()))
    B = _TRIC.astype(np.float64)
    p = s.pos.astype(np.float64)
    d = p[None, :, :] - p[:, None, :]
    best = np.full(d.shape[:2], np.inf)
    for i in range(-2, 3):
        for j in range(-2, 3):
            for k in range(-2, 3):
                best = np.minimum(best, np.linalg.norm(d + i * B[0] + j * B[1] + k * B[2], axis=-1))
    np.fill_diagonal(best, np.inf)
    want = set(zip(*np.nonzero(best < rc - 1e-4)))
    unsure = set(zip(*np.nonzero(np.abs(best - rc) <= 1e-4)))
    assert want <= got and got <= want | unsure
    assert len(want) > 1000


def test_triclinic_energy_is_lattice_periodic():
    # moving every atom by a lattice vector changes nothing but float32
    # rounding of the positions
    s = w.triclinic_system(200, _TRIC, seed=3)
    at, mt = w.aev_table(4), w.mlp_table(4)
    r0 = o.energy_forces(s, aev_table=at, mlp_table=mt)
    moved = (s.pos.astype(np.float64) + _TRIC[1] - _TRIC[2]).astype(np.float32)
    r1 = o.energy_forces(moved, s.species, s.mol_offsets, _TRIC, aev_table=at, mlp_table=mt)
    np.testing.assert_allclose(r1.E, r0.E, rtol=1e-5)
    assert np.linalg.norm(r1.F - r0.F) <= 1e-4 * np.linalg.norm(r0.F)


def test_triclinic_box_checks():
    from oracle.neighbors import check_triclinic
    check_triclinic(_TRIC, 5.1)
    for bad in ([[16, 1, 0], [3, 15, 0], [-4, 5, 14]],     # a not along x
                [[16, 0, 0], [9, 15, 0], [-4, 5, 14]],     # |bx| > ax/2
                [[16, 0, 0], [3, 15, 0], [-4, 5, 9.0]]):   # narrower than 2 rc
        with pytest.raises(ValueError):
            check_triclinic(np.array(bad, dtype=np.float32), 5.1)


def test_neighborhood_reference_equals_whole_system():
    """The per-atom force from the oracle on an atom's neighborhood (used by
    the sampled GPU test of the 23,001-atom box) equals the whole-system
    oracle force on the 1,500-water box: the force on an atom depends only
    on the energies of the atom and its radial neighbors."""
    from neighborhood import neighborhood_reference
    s = w.config_system(2)
    at, mt = w.aev_table(4), w.mlp_table(4)
    full = o.energy_forces(s, aev_table=at, mlp_table=mt)
    I, J = pair_list(s.pos, s.mol_offsets, s.box, at.rc_rad)
    for k in (0, 17, 1234, 4499):
        Fk, nset = neighborhood_reference(s, at, mt, k)
        np.testing.assert_allclose(Fk, full.F[k], rtol=1e-12, atol=1e-12)
        assert nset == set(J[I == k].tolist())
