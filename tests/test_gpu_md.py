"""GPU molecular dynamics and serving against the oracle integrator.

Bars: velocity Verlet on the GPU tracks the FP64 oracle integrator to
|dx| <= 1e-6 A over 20 steps (FP32 forces at FP32-rounded positions on both
sides); time reversal returns within 1e-5 A; a served request equals the same
molecule integrated alone to |dx| <= 1e-4 A and relative energy 1e-5 after
its steps (the only difference is the order of atomic force additions).
"""
import numpy as np
import pytest
import torch

import oracle as o
import workloads as w
from gpu_util import potential, to_dev

pytestmark = pytest.mark.gpu


def announce(msg):
    print(f"\n[case] {msg}", flush=True)


def _md_gpu(pot, s, v0, dt, n_steps):
    pos, sp, off = to_dev(s)
    x = torch.from_numpy(s.pos.astype(np.float64)).cuda()
    v = torch.from_numpy(v0).cuda()
    m = torch.from_numpy(w.MASS_AMU[s.species]).cuda()
    _, F = pot.energy_forces(pos, sp, off, s.box)
    Ep, Ek = pot.md_steps(x, v, F, m, sp, off, dt, n_steps, s.box)
    pot.check()
    return x.cpu().numpy(), v.cpu().numpy(), Ep.cpu().numpy(), Ek.cpu().numpy()


def test_velocity_verlet_matches_oracle():
    s = w.single_molecule(24, seed=5, n_species=4)
    announce("md vs oracle integrator, 24 atoms, 20 steps")
    pot, at, mt = potential(4, "fp32")
    v0 = w.maxwell_boltzmann(s.species, 300.0, np.random.default_rng(1))
    x, v, Ep, Ek = _md_gpu(pot, s, v0, 0.5, 20)

    def ff(x32):
        r = o.energy_forces(x32, s.species, s.mol_offsets, None, aev_table=at, mlp_table=mt)
        return r.E, r.F

    xo, vo, rec = o.velocity_verlet(s.pos.astype(np.float64), v0, w.MASS_AMU[s.species], ff, 0.5, 20)
    print(f"max|dx| {np.abs(x - xo).max():.2e}  max|dv| {np.abs(v - vo).max():.2e}")
    assert np.abs(x - xo).max() <= 1e-6
    assert np.abs(v - vo).max() <= 1e-7
    assert abs(Ek[0] - rec[-1][2]) <= 1e-6 * abs(rec[-1][2])
    assert abs(Ep[0] - rec[-1][1]) <= 1e-5 * max(1.0, abs(rec[-1][1]))


def test_time_reversibility():
    s = w.single_molecule(40, seed=6, n_species=7)
    announce("md time reversal, 40 atoms")
    pot, at, mt = potential(7, "fp32")
    v0 = w.maxwell_boltzmann(s.species, 300.0, np.random.default_rng(2))
    x1, v1, _, _ = _md_gpu(pot, s, v0, 0.5, 50)
    s1 = w.System(x1.astype(np.float32), s.species, s.mol_offsets, None, 7)
    # continue from the FP64 state, reversed
    pos, sp, off = to_dev(s1)
    x = torch.from_numpy(x1).cuda()
    v = torch.from_numpy(-v1).cuda()
    m = torch.from_numpy(w.MASS_AMU[s.species]).cuda()
    _, F = pot.energy_forces(x.float(), sp, off, None)
    pot.md_steps(x, v, F, m, sp, off, 0.5, 50)
    pot.check()
    err = np.abs(x.cpu().numpy() - s.pos.astype(np.float64)).max()
    print(f"reversal max|dx| {err:.2e}")
    assert err <= 1e-5


def test_nve_energy_error_matches_oracle_integrator():
    # The random-weight potential heats a water box quickly (kinetic energy
    # grows ~20x in 100 fs), so energy conservation is checked against the FP64
    # oracle integrator on the same system and step: the GPU path's
    # max |E_tot - E_0| must be no worse than the oracle's, up to a small
    # FP32 allowance.
    s = w.water_box(60, 12.0, seed=12, n_species=7)
    announce(f"NVE energy error vs oracle, {s.n_atoms}-atom water box, 160 steps at 0.25 fs")
    pot, at, mt = potential(7, "fp32")
    v0 = w.maxwell_boltzmann(s.species, 300.0, np.random.default_rng(3))
    pos, sp, off = to_dev(s)
    x = torch.from_numpy(s.pos.astype(np.float64)).cuda()
    v = torch.from_numpy(v0).cuda()
    m = torch.from_numpy(w.MASS_AMU[s.species]).cuda()
    E0, F = pot.energy_forces(pos, sp, off, s.box)
    tot = [E0.item() + o.kinetic_energy(v0, w.MASS_AMU[s.species])]
    for _ in range(16):
        Ep, Ek = pot.md_steps(x, v, F, m, sp, off, 0.25, 10, s.box)
        tot.append(Ep.item() + Ek.item())
    pot.check()
    gpu_err = np.abs(np.array(tot) - tot[0]).max() / s.n_atoms

    def ff(x32):
        r = o.energy_forces(x32, s.species, s.mol_offsets, s.box, aev_table=at, mlp_table=mt)
        return r.E, r.F

    _, _, rec = o.velocity_verlet(s.pos.astype(np.float64), v0, w.MASS_AMU[s.species], ff, 0.25,
                                  160, record_every=10)
    e = np.array([r[1] + r[2] for r in rec])
    ora_err = np.abs(e - e[0]).max() / s.n_atoms
    print(f"max |E_tot - E_0| / atom: GPU {gpu_err:.3e} eV, oracle {ora_err:.3e} eV")
    assert gpu_err <= 1.2 * ora_err + 1e-5


def _requests(n, seed=3):
    """n requests with step counts 20..40, so requests finish in different
    rounds and survivors share launches with newly admitted ones."""
    reqs = w.poisson_requests(n, rate=1000.0, seed=seed, n_steps=30)
    for r in reqs:
        r.n_steps = 20 + (7 * r.req_id) % 21
    return reqs


def _serve_staggered(srv, reqs, n_first=6, every=3):
    """Submits the first n_first requests, then one more every `every`
    rounds while the server runs; returns the delivered results and the
    server statistics."""
    def submit(r):
        assert srv.submit(r.req_id, r.system.pos.astype(np.float64), r.vel, r.system.species,
                          r.n_steps) == 0
    for r in reqs[:n_first]:
        submit(r)
    nxt = n_first
    done = {}
    rounds = 0
    while len(done) < len(reqs):
        if nxt < len(reqs) and rounds % every == 0:
            submit(reqs[nxt])
            nxt += 1
        srv.step()
        rounds += 1
        for i in srv.poll():
            done[i] = srv.result(i, reqs[i].system.n_atoms)
        assert rounds < 5000
    st = srv.stats()
    print(f"{rounds} rounds; stats {st}")
    # survivors and new admissions in one repack, and requests at different
    # steps of their trajectories in one launch
    assert st["mixed_rounds"] >= 1
    assert st["max_phases_per_launch"] >= 2
    return done, st


def test_serving_alone_equals_mix():
    from paper_2310_03121_amd import Server
    announce("server: continuous batching vs each request alone")
    pot, at, mt = potential(7, "fp32")
    reqs = _requests(24)
    srv = Server(pot, hbm_budget_bytes=8 << 30, max_atoms=900, max_mols=12, dt_fs=0.5,
                 mass_amu=w.MASS_AMU)
    done, st = _serve_staggered(srv, reqs)
    worst = 0.0
    for r in reqs[:10]:
        x, v, Ep, Ek = _md_gpu(pot, r.system, r.vel, 0.5, r.n_steps)
        d = done[r.req_id]
        dx = np.abs(d["x"] - x).max()
        worst = max(worst, dx)
        assert dx <= 1e-4, (r.req_id, dx)
        assert abs(d["e_pot"] - Ep[0]) <= 1e-5 * max(1.0, abs(Ep[0]))
        assert abs(d["e_kin"] - Ek[0]) <= 1e-5 * max(1.0, abs(Ek[0]))
        assert d["t_submit"] <= d["t_admit"] <= d["t_done"]
    print(f"alone vs mix: worst max|dx| {worst:.2e} A")


def _serve_all(srv, reqs):
    ids = []
    for r in reqs:
        code = srv.submit(r.req_id, r.system.pos.astype(np.float64), r.vel, r.system.species,
                          r.n_steps)
        assert code in (0, 9)  # 9: larger than the server can ever hold
        if code == 0:
            ids.append(r.req_id)
    got = set()
    rounds = 0
    while len(got) < len(ids):
        srv.step()
        rounds += 1
        got.update(srv.poll())
        assert rounds < 20000
    return ids, rounds, srv.stats()


def test_serving_respects_capacity_and_budget():
    from paper_2310_03121_amd import Server
    announce("server: tiny HBM budget admits fewer atoms at once")
    pot, at, mt = potential(7, "fp32")
    reqs = _requests(8, seed=9)
    big = max(r.system.n_atoms for r in reqs)
    small = Server(pot, hbm_budget_bytes=24 << 20, max_atoms=4096, max_mols=64, dt_fs=0.5,
                   mass_amu=w.MASS_AMU)
    ids, rounds, st = _serve_all(small, reqs)
    free = Server(pot, hbm_budget_bytes=8 << 30, max_atoms=4096, max_mols=64, dt_fs=0.5,
                  mass_amu=w.MASS_AMU)
    ids_f, rounds_f, st_f = _serve_all(free, reqs)
    print(f"24 MiB budget: {len(ids)} requests, {rounds} rounds, {st}; "
          f"8 GiB: {rounds_f} rounds, {st_f} (largest request {big} atoms)")
    # the budget lowered the capacity, and with it the atoms on the device at
    # once, which stretched the same work over more rounds
    assert st["capacity_atoms"] < 4096 and st_f["capacity_atoms"] == 4096
    assert st["peak_atoms"] <= st["capacity_atoms"]
    assert st["peak_atoms"] < st_f["peak_atoms"]
    assert rounds > rounds_f
    # exactly the requests that fit the capacity were accepted
    assert ids == [r.req_id for r in reqs if r.system.n_atoms <= st["capacity_atoms"]]


def test_device_errors_reach_md_and_served_requests():
    """A neighbor capacity of 16 with molecules denser than that: the
    overflow bit raised during an MD segment is reported by nnp_check after
    nnp_md_steps, and by nnp_server_result for every served request that was
    on the device while it was raised."""
    from paper_2310_03121_amd import NNPError, Server
    announce("device status: capacity overflow in md_steps and in serving")
    pot, at, mt = potential(7, "fp32", max_neighbors=16)
    # a liquid-density cluster (atoms of the 1,500-water box within 6 A of its
    # centre) as one molecule without a box: about 50 neighbors per atom
    wb = w.config_system(2)
    keep = np.nonzero(np.linalg.norm(wb.pos - wb.pos.mean(0), axis=1) < 6.0)[0]
    s = w.System(wb.pos[keep].copy(), wb.species[keep].copy(),
                 np.array([0, keep.size], np.int32), None, 7)
    pos, sp, off = to_dev(s)
    v0 = w.maxwell_boltzmann(s.species, 300.0, np.random.default_rng(1))
    x = torch.from_numpy(s.pos.astype(np.float64)).cuda()
    v = torch.from_numpy(v0).cuda()
    m = torch.from_numpy(w.MASS_AMU[s.species]).cuda()
    _, F = pot.energy_forces(pos, sp, off, None)
    with pytest.raises(NNPError) as e:
        pot.check()
    assert e.value.code == 4
    pot.md_steps(x, v, F, m, sp, off, 0.5, 5, None)
    with pytest.raises(NNPError) as e:
        pot.check()
    assert e.value.code == 4
    srv = Server(pot, hbm_budget_bytes=1 << 30, max_atoms=512, max_mols=8, dt_fs=0.5,
                 mass_amu=w.MASS_AMU)
    assert srv.submit(0, s.pos.astype(np.float64), v0, s.species, 4) == 0
    got = []
    rounds = 0
    while not got:
        srv.step()
        got = srv.poll()
        rounds += 1
        assert rounds < 100
    assert srv.result(0, s.n_atoms, check=False)["status"] == 4
    with pytest.raises(NNPError):
        srv.result(0, s.n_atoms)


# ------------------------------------------------------- LF-Middle Langevin
def test_langevin_matches_oracle():
    s = w.single_molecule(24, seed=5, n_species=4)
    announce("LF-Middle Langevin vs oracle, 24 atoms, 20 steps, 300 K, 50/ps")
    pot, at, mt = potential(4, "fp32")
    v0 = w.maxwell_boltzmann(s.species, 300.0, np.random.default_rng(1))
    pos, sp, off = to_dev(s)
    x = torch.from_numpy(s.pos.astype(np.float64)).cuda()
    v = torch.from_numpy(v0.copy()).cuda()
    m = torch.from_numpy(w.MASS_AMU[s.species]).cuda()
    _, F = pot.energy_forces(pos, sp, off, None)
    Ep, Ek = pot.langevin_steps(x, v, F, m, sp, off, 0.5, 20, 300.0, 50.0, seed=2024)
    pot.check()

    def ff(x32):
        r = o.energy_forces(x32, s.species, s.mol_offsets, None, aev_table=at, mlp_table=mt)
        return r.E, r.F

    xo, vo, rec = o.langevin_middle(s.pos.astype(np.float64), v0, w.MASS_AMU[s.species], ff,
                                    0.5, 20, 300.0, 50.0, seed=2024)
    dx = np.abs(x.cpu().numpy() - xo).max()
    dv = np.abs(v.cpu().numpy() - vo).max()
    print(f"max|dx| {dx:.2e}  max|dv| {dv:.2e}  KE {Ek.item():.4f} vs {rec[-1][2]:.4f}")
    assert dx <= 1e-6 and dv <= 1e-6
    assert abs(Ek.item() - rec[-1][2]) <= 1e-5 * abs(rec[-1][2])
    assert abs(Ep.item() - rec[-1][1]) <= 1e-5 * max(1.0, abs(rec[-1][1]))


def test_langevin_split_calls_draw_the_same_noise():
    s = w.single_molecule(40, seed=6, n_species=7)
    announce("Langevin 20 steps in one call vs 10 + 10")
    pot, at, mt = potential(7, "fp32")
    v0 = w.maxwell_boltzmann(s.species, 300.0, np.random.default_rng(2))
    pos, sp, off = to_dev(s)
    m = torch.from_numpy(w.MASS_AMU[s.species]).cuda()
    res = []
    for split in ((20,), (10, 10)):
        x = torch.from_numpy(s.pos.astype(np.float64)).cuda()
        v = torch.from_numpy(v0.copy()).cuda()
        _, F = pot.energy_forces(pos, sp, off, None)
        k0 = 0
        for nstep in split:
            pot.langevin_steps(x, v, F, m, sp, off, 0.5, nstep, 300.0, 5.0, seed=99, step0=k0)
            k0 += nstep
        pot.check()
        res.append((x.cpu().numpy(), v.cpu().numpy()))
    # the same draws: only the order of the FP32 force atomics differs
    # (a different draw would move atoms by ~1e-2 A)
    assert np.abs(res[0][0] - res[1][0]).max() <= 1e-7
    assert np.abs(res[0][1] - res[1][1]).max() <= 1e-7


def test_langevin_full_friction_draws_the_temperature():
    # c = exp(-friction dt) ~ 0: after one step every velocity is a fresh
    # Maxwell-Boltzmann draw, so 2 KE / (3 N kB) estimates T
    s = w.config_system(2)
    announce(f"Langevin thermalization, {s.n_atoms}-atom water box")
    pot, at, mt = potential(4, "fp32")
    pos, sp, off = to_dev(s)
    x = torch.from_numpy(s.pos.astype(np.float64)).cuda()
    v = torch.zeros((s.n_atoms, 3), dtype=torch.float64, device="cuda")
    m = torch.from_numpy(w.MASS_AMU[s.species]).cuda()
    _, F = pot.energy_forces(pos, sp, off, s.box)
    for T in (300.0, 77.0):
        _, Ek = pot.langevin_steps(x, v, F, m, sp, off, 0.5, 1, T, 1e6, seed=5, step0=int(T),
                                   box=s.box)
        pot.check()
        T_est = 2 * Ek.item() / (3 * s.n_atoms * o.integrator.KB_EV)
        print(f"T {T}: estimate {T_est:.2f}")
        assert abs(T_est / T - 1) < 5 * np.sqrt(2.0 / (3 * s.n_atoms))


def test_serving_langevin_alone_equals_mix():
    # each request's noise is keyed by its id and counted by its own atoms
    # and steps: inside the batch it follows the same trajectory as the same
    # molecule integrated alone with nnp_langevin_steps(seed=id)
    from paper_2310_03121_amd import Server
    announce("server, LF-Middle Langevin: batch vs each request alone")
    pot, at, mt = potential(7, "fp32")
    reqs = _requests(16, seed=4)
    srv = Server(pot, hbm_budget_bytes=8 << 30, max_atoms=700, max_mols=10, dt_fs=0.5,
                 mass_amu=w.MASS_AMU)
    srv.set_langevin(300.0, 20.0)
    done, st = _serve_staggered(srv, reqs, n_first=4, every=4)
    worst = 0.0
    for r in reqs[:8]:
        s = r.system
        pos, sp, off = to_dev(s)
        x = torch.from_numpy(s.pos.astype(np.float64)).cuda()
        v = torch.from_numpy(r.vel.copy()).cuda()
        m = torch.from_numpy(w.MASS_AMU[s.species]).cuda()
        _, F = pot.energy_forces(pos, sp, off, None)
        Ep, Ek = pot.langevin_steps(x, v, F, m, sp, off, 0.5, r.n_steps, 300.0, 20.0,
                                    seed=r.req_id)
        pot.check()
        d = done[r.req_id]
        dx = np.abs(d["x"] - x.cpu().numpy()).max()
        worst = max(worst, dx)
        assert dx <= 1e-4, (r.req_id, dx)
        assert abs(d["e_pot"] - Ep.item()) <= 1e-5 * max(1.0, abs(Ep.item()))
        assert abs(d["e_kin"] - Ek.item()) <= 1e-5 * max(1.0, abs(Ek.item()))
    print(f"Langevin alone vs mix: worst max|dx| {worst:.2e} A")


def test_serving_delivers_more_than_one_poll_batch_at_once():
    # 1,100 small requests admitted together finish in the same round: every
    # one of them is delivered, although the library hands ids out 1,024 per
    # poll call
    from paper_2310_03121_amd import Server
    announce("server: 1,100 requests finishing in one round")
    pot, _, _ = potential(4, "bf16", max_neighbors=64)
    srv = Server(pot, hbm_budget_bytes=2 << 30, max_atoms=16384, max_mols=2048, dt_fs=0.5,
                 mass_amu=w.MASS_AMU)
    mol = w.single_molecule(8, seed=9, n_species=4)
    v0 = np.zeros((8, 3))
    for k in range(1100):
        assert srv.submit(k, mol.pos.astype(np.float64), v0, mol.species, 2) == 0
    got = []
    for _ in range(20):
        srv.step()
        got += srv.poll()
        if len(got) == 1100:
            break
    assert sorted(got) == list(range(1100))
    assert srv.active == 0 and srv.pending == 0
    r0, r1 = srv.result(0, 8), srv.result(1099, 8)
    # same molecule, same start: the same trajectory up to force-summation order
    assert np.abs(r0["x"] - r1["x"]).max() <= 1e-8
