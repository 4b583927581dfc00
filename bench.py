"""Benchmark: energy + force evaluations of the symmetry-function potential.

One step = one pass of the whole path (staging and species sort, neighbor
search, symmetry functions, per-element networks, FP64 energy sums, network
adjoint, symmetry-function adjoint and force scatter) over one batch.

Default workload: 512 conformations x 64 atoms (32,768 atoms), seven
elements, 1008 features, networks 1008-256-192-160-1, no box; inputs resident
in HBM before the timed region.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--workload batch|water1500|water7667]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "atoms·evals/s (E+F), BF16 vs FP32 path at fixed force error; p99 req latency"
PEAK_TFLOPS = {"bf16": 2500.0, "fp32": 157.3}   # MI355X dense MFMA
PEAK_HBM_GBS = 8000.0


_T0 = time.perf_counter()


def progress(msg):
    """One line per finished leg on stderr (stdout carries only the result)."""
    print(f"[bench {time.perf_counter() - _T0:7.1f} s] {msg}", file=sys.stderr, flush=True)


def mlp_flops_per_atom(widths, F):
    w = list(widths)
    w[0] = F
    fwd = sum(2 * w[l] * w[l + 1] for l in range(len(w) - 1))
    bwd = sum(2 * w[l] * w[l + 1] for l in range(len(w) - 2))  # input-gradient chain
    return fwd, bwd


def stage_flops(widths, F):
    """Algorithmic FLOPs per atom of each network stage."""
    w1, w2, w3 = widths[1], widths[2], widths[3]
    d = {
        "mlp_layer1": 2 * F * w1, "mlp_layer2": 2 * w1 * w2, "mlp_layer3_head": 2 * w2 * w3 + 2 * w3,
        "mlp_bwd_layer3": 2 * w3 * w2, "mlp_bwd_layer2": 2 * w2 * w1, "mlp_bwd_dEdG": 2 * w1 * F,
    }
    d["mlp_mid_fused"] = (d["mlp_layer2"] + d["mlp_layer3_head"] + d["mlp_bwd_layer3"]
                          + d["mlp_bwd_layer2"])
    d["mlp_net_fused"] = d["mlp_layer1"] + d["mlp_mid_fused"] + d["mlp_bwd_dEdG"]
    return d


# Algorithmic fp32 operations of the symmetry-function kernels (add, mul, FMA
# and each transcendental counted as one lane operation), from the radial and
# angular terms as
# defined: per radial neighbor pair 16 shifts x 6 (difference, square, scale,
# exp, cutoff product, sum) + 11 (distance, cutoff); per angular triple 151
# (cosine 7, kappa and sine 4, 8 angle shifts x 7, 4 distance shifts x 4 + 2,
# 32 products and sums, cutoff product 2).  The adjoint recomputes the forward
# terms and adds their derivatives and the scatter: 199 per radial pair, 280
# per angular triple.
AEV_OPS = {"aev_fwd": (107, 151), "aev_bwd_forces": (199, 280)}
# Lane operations per second of the FP32 vector units: 1,024 SIMDs x 32 lanes
# per clock x 2.4 GHz (one add, multiply, FMA or transcendental per lane and
# clock); the same rate is the 157.3 TFLOP/s FP32 vector peak with an FMA
# counted as 2.  The FMA issue loop measures about 61 % of it.
PEAK_VALU_TOPS = 78.6


def pair_counts(pot, n_atoms):
    """Directed radial pairs and angular triples of the last evaluation."""
    counts, _ = pot.debug_neighbors(n_atoms)
    c = counts.cpu().numpy().astype(np.int64)
    return int(c[:, 0].sum()), int((c[:, 1] * (c[:, 1] - 1) // 2).sum())


def source_digest():
    """sha256 over the HIP sources and headers of the library."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2310_03121_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".h")):
            h.update(f.encode())
            h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()


def profiled_traffic(stage, workload_key):
    """HBM bytes per launch of `stage` from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE scaled against a copy of known size), or None
    when the summary is missing or was taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload_key}.md")
    if not os.path.exists(path):
        return None
    digest, rows = None, {}
    for line in open(path):
        if line.startswith("source_digest:"):
            digest = line.split(":", 1)[1].strip()
        elif line.startswith("|") and not line.startswith("|--"):
            cells = [c.strip() for c in line.strip().strip("|").split("|")]
            if len(cells) >= 6 and cells[0] != "stage":
                try:
                    rows[cells[0]] = float(cells[5])
                except ValueError:
                    pass
    if digest != source_digest() or stage not in rows:
        return None
    return rows[stage]


def profiled_kernel_ms(stage, workload_key):
    """Mean duration (ms) of the stage's kernel in the committed rocprofv3
    kernel-trace summary, or None when missing or taken on other sources."""
    path = os.path.join(ROOT, "profiles", f"kernels_{workload_key}.md")
    if not os.path.exists(path):
        return None
    digest, hit = None, None
    for line in open(path):
        if line.startswith("source_digest:"):
            digest = line.split(":", 1)[1].strip()
        elif line.startswith("|") and not line.startswith("|--"):
            cells = [c.strip() for c in line.strip().strip("|").split("|")]
            if len(cells) >= 4 and cells[0] == stage and hit is None:
                try:
                    hit = float(cells[3]) * 1e-3
                except ValueError:
                    pass
    if digest != source_digest():
        return None
    return hit


def profiled_valu(stage, workload_key):
    """(wave64 VALU instructions per wavefront, wavefronts per launch) of the
    stage's kernel from the committed instruction-counter summary, or None
    when it is missing or was taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", f"sq_counters_{workload_key}.md")
    if not os.path.exists(path):
        return None
    digest, hit = None, None
    for line in open(path):
        if line.startswith("source_digest:"):
            digest = line.split(":", 1)[1].strip()
        elif line.startswith("|") and not line.startswith("|--"):
            cells = [c.strip() for c in line.strip().strip("|").split("|")]
            # the first table's row (a later table of the file holds MFMA counts)
            if len(cells) >= 4 and cells[0] == stage and hit is None:
                try:
                    hit = (float(cells[3]), float(cells[2]))
                except ValueError:
                    pass
    if digest != source_digest():
        return None
    return hit


WORKLOAD_KEYS = {"batch": "batch512x64", "water1500": "water1500", "water7667": "water7667",
                 "mol24": "mol24"}
# Neighbor-list capacity per atom (the handle's max_neighbors): the batch's
# longest list is 14 entries, the water boxes' 71.  Overflow is detected on
# the device and reported, never silently truncated.
MAX_NEIGHBORS = {"batch": 64, "water1500": 128, "water7667": 128, "mol24": 64}


def workload(name):
    import workloads as w
    if name == "batch":
        return w.config_system(1), 7, "512 conformations x 64 atoms, 7 elements, 1008 features, no box"
    if name == "water1500":
        return w.config_system(2), 4, "1,500-water box (4,500 atoms), L=35.5 A, 4 elements, 384 features"
    if name == "water7667":
        return w.config_system(4), 7, "7,667-water box (23,001 atoms), L=61.2 A, 7 elements, 1008 features"
    if name == "mol24":
        return w.config_system(0), 4, "one 24-atom molecule, 4 elements, 384 features, no box"
    raise SystemExit(f"unknown workload {name}")


def time_path(pot, pos, sp, off, box, steps, warmup):
    import torch
    out = (torch.empty(off.shape[0] - 1, dtype=torch.float64, device=pos.device),
           torch.empty((pos.shape[0], 3), dtype=torch.float32, device=pos.device))
    for _ in range(warmup):
        pot.energy_forces(pos, sp, off, box, out=out)
    pot.check()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        pot.energy_forces(pos, sp, off, box, out=out)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    pot.check()
    # the same evaluations replayed from a captured HIP graph
    g = pot.capture(pos, sp, off, box)
    for _ in range(warmup):
        g.launch()
    g.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g.launch()
    g.synchronize()
    dt_graph = time.perf_counter() - t0
    g.check()
    del g
    # per-stage device times with HIP events on the launch stream, same steps
    pot.profile(True)
    for _ in range(steps):
        pot.energy_forces(pos, sp, off, box, out=out)
        pot.profile_collect()
    stages = pot.profile_read()
    pot.profile(False)
    return dt, dt_graph, out, stages


def backward_leg(pot, pos, sp, off, box, steps, warmup, mt):
    """nnp_backward on the workload: the whole forward pass, dL/dpos (the
    forces' adjoint) and every weight gradient for L = sum_m E_m, timed like
    the evaluation, with the weight-gradient stage's own device time and its
    algorithmic MFMA rate (2 FLOP per multiply-add of dW = delta^T h over all
    atoms and layers)."""
    import torch
    n, nmol = pos.shape[0], off.shape[0] - 1
    dLdE = torch.ones(nmol, dtype=torch.float64, device=pos.device)
    for _ in range(warmup):
        pot.backward(pos, sp, off, dLdE, box=box)
    pot.check()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        pot.backward(pos, sp, off, dLdE, box=box)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    pot.check()
    pot.profile(True)
    for _ in range(steps):
        pot.backward(pos, sp, off, dLdE, box=box)
        pot.profile_collect()
    stages = pot.profile_read()
    pot.profile(False)
    st = {k: v[0] / max(v[1], 1) for k, v in stages.items() if v[1]}
    w = list(mt.widths)
    wg_flop = 2 * n * sum(w[l] * w[l + 1] for l in range(len(w) - 1))
    wg_ms = st.get("weight_grads")
    return {"ms_per_call": 1e3 * dt / steps, "atoms_per_s": n * steps / dt,
            "stages_ms": st, "weight_grad_flop": wg_flop,
            "weight_grad_tflops": wg_flop / (wg_ms * 1e-3) / 1e12 if wg_ms else None}


def latency_leg(pot, pos, sp, off, box, n_evals=1000, warmup=50):
    """Per-evaluation latency: each captured evaluation is launched and waited
    for on its own (median and p99 over n_evals, after warm-up)."""
    g = pot.capture(pos, sp, off, box)
    for _ in range(warmup):
        g.launch()
    g.synchronize()
    lat = np.empty(n_evals)
    for k in range(n_evals):
        t0 = time.perf_counter()
        g.launch()
        g.synchronize()
        lat[k] = time.perf_counter() - t0
    g.check()
    del g
    return {"evals": n_evals, "warmup": warmup, "median_us": float(np.median(lat) * 1e6),
            "p99_us": float(np.percentile(lat, 99) * 1e6), "launch": "graph replay, synchronized"}


def relax(pot, x, sp, off, box, md, n_iter=400, dt=0.25, dt_max=1.0, max_step=0.05):
    """FIRE energy minimization (Bitzek et al., PRL 97, 170201, 2006) of the
    float64 positions x with the GPU forces: the random-weight potential is
    far from equilibrium at the generated geometry, and NVE from there turns
    that potential energy into heat.  Returns energy and largest force before
    and after."""
    import torch
    acc = 9.648533e-3
    v = torch.zeros_like(x)
    alpha, n_pos = 0.1, 0
    E, F = pot.energy_forces(x.float(), sp, off, box)
    e0, f0 = E.sum().item(), F.norm(dim=1).max().item()
    for _ in range(n_iter):
        Fd = F.double()
        p = float((Fd * v).sum())
        if p > 0.0:
            fn, vn = Fd.norm(), v.norm()
            v = (1 - alpha) * v + alpha * vn * Fd / fn.clamp_min(1e-30)
            n_pos += 1
            if n_pos > 5:
                dt, alpha = min(dt * 1.1, dt_max), alpha * 0.99
        else:
            v.zero_()
            dt, alpha, n_pos = dt * 0.5, 0.1, 0
        v += dt * acc * Fd / md[:, None]
        step = dt * v
        scale = (max_step / step.norm(dim=1).max().clamp_min(1e-30)).clamp(max=1.0)
        x += step * scale
        if box is not None:
            L = torch.tensor(np.asarray(box, np.float64), device=x.device)
            x -= L * torch.floor(x / L)
        E, F = pot.energy_forces(x.float(), sp, off, box)
    pot.check()
    return {"iterations": n_iter, "E_eV_before_after": [e0, E.sum().item()],
            "max_force_eV_per_A_before_after": [f0, F.norm(dim=1).max().item()]}


def nve_leg(pot, s, n_steps=1000, dt=0.5, every=10, seed=4, relax_iters=0):
    """NVE velocity Verlet from Maxwell-Boltzmann velocities at 300 K
    (optionally after a FIRE relaxation of the generated geometry): total
    energy sampled every `every` steps; drift is the least-squares slope of
    E_tot(t), plus the largest excursion from the first sample, both per atom."""
    import torch
    import workloads as w
    dev = torch.device("cuda:0")
    m = w.MASS_AMU[s.species]
    v0 = w.maxwell_boltzmann(s.species, 300.0, np.random.default_rng(seed))
    x = torch.from_numpy(s.pos.astype(np.float64)).to(dev)
    v = torch.from_numpy(v0).to(dev)
    md = torch.from_numpy(m).to(dev)
    sp = torch.from_numpy(s.species).to(dev)
    off = torch.from_numpy(s.mol_offsets).to(dev)
    relaxed = relax(pot, x, sp, off, s.box, md, n_iter=relax_iters) if relax_iters else None
    E0, F = pot.energy_forces(x.float(), sp, off, s.box)
    # E_tot as the integrator reports it (potential + kinetic after each
    # chunk of steps); the series starts after the first chunk
    t, tot, ek = [], [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(n_steps // every):
        Ep, Ek = pot.md_steps(x, v, F, md, sp, off, dt, every, s.box)
        t.append((k + 1) * every * dt)
        tot.append(float(Ep.sum().item()) + float(Ek.sum().item()))
        ek.append(float(Ek.sum().item()))
    wall = time.perf_counter() - t0
    pot.check()
    t = np.array(t) * 1e-3  # ps
    e = (np.array(tot) - tot[0]) * 1e3 / s.n_atoms  # meV per atom
    slope = float(np.polyfit(t, e, 1)[0])
    return {"steps": n_steps, "dt_fs": dt, "sample_every": every, "relaxation": relaxed,
            "drift_meV_per_ps_per_atom": slope, "max_abs_dev_meV_per_atom": float(np.abs(e).max()),
            "kinetic_energy_eV_first_last_sample": [ek[0], ek[-1]],
            "kinetic_energy_eV_max_sample": float(np.max(ek)),
            "ms_per_step": wall * 1e3 / n_steps}


def ensemble_leg(s, at, S, args, single):
    """The same workload with an ensemble of M networks (seeds 101.. for 7
    elements, 100.. for 4): mean energy and forces, one neighbor search and
    one symmetry-function pass per evaluation.  Reports the time per
    evaluation and its ratio to the single network measured above (the
    ensemble's parity with the FP64 oracle is a GPU test)."""
    progress("importing torch")
    import torch
    import workloads as w
    from paper_2310_03121_amd import Potential
    progress("imports done")
    M = args.ensemble
    base = 101 if S == 7 else 100
    members = [w.mlp_table(S, seed=base + k) for k in range(M)]
    dev = torch.device("cuda:0")
    pos = torch.from_numpy(s.pos).to(dev)
    sp = torch.from_numpy(s.species).to(dev)
    off = torch.from_numpy(s.mol_offsets).to(dev)
    out = {"members": M}
    for prec in single:
        pot = Potential.ensemble_from_tables(at, members, precision=prec,
                                             max_neighbors=MAX_NEIGHBORS[args.workload])
        dt_e, dt_g, (E, F), _ = time_path(pot, pos, sp, off, s.box, args.steps, args.warmup)
        dt = min(dt_e, dt_g)
        r = {"ms_per_step": 1e3 * dt / args.steps, "value": s.n_atoms * args.steps / dt,
             "ratio_to_single": (1e3 * dt / args.steps) / single[prec]["ms_per_step"]}
        out[prec] = r
        del pot
        torch.cuda.empty_cache()
    return out


def ceilings():
    """Device ceilings measured here: a large device copy, large square GEMMs
    (hipBLASLt through torch) in BF16 and FP32, and library GEMMs at the
    network's own layer shapes for comparison with the fused kernels."""
    import torch

    def timed(fn, reps):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps * 1e-3  # s

    out = {}
    src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    dt = timed(lambda: dst.copy_(src), 20)
    out["copy_GBps"] = 2 * src.numel() / dt / 1e9
    del src, dst
    for dtype, name, n in ((torch.bfloat16, "bf16", 8192), (torch.float32, "fp32", 8192)):
        a = torch.randn(n, n, device="cuda", dtype=dtype)
        b = torch.randn(n, n, device="cuda", dtype=dtype)
        dt = timed(lambda: a @ b, 10)
        out[f"gemm_{name}_{n}^3_TFLOPs"] = 2 * n ** 3 / dt / 1e12
        del a, b
    shapes = []
    for M, K, N in ((32768, 1024, 256), (32768, 256, 192), (32768, 192, 160), (32768, 160, 192),
                    (32768, 192, 256), (32768, 256, 1024)):
        a = torch.randn(M, K, device="cuda", dtype=torch.bfloat16)
        b = torch.randn(K, N, device="cuda", dtype=torch.bfloat16)
        dt = timed(lambda: a @ b, 30)
        shapes.append({"M": M, "K": K, "N": N, "us": dt * 1e6})
        del a, b
    out["library_bf16_gemm_at_layer_shapes"] = shapes
    torch.cuda.empty_cache()
    return out


CEILING_KINDS = {"mfma_bf16": 0, "mfma_fp32": 1, "valu_fma_fp32": 2, "valu_exp2_fp32": 3}


def issue_ceilings():
    """Compute ceilings measured on this device by the issue loops of
    libnnp_ceilings.so (eight independent chains per wave, 8 waves per CU):
    BF16 and FP32 MFMA (TFLOP/s), FP32 FMA (TFLOP/s, an FMA counting 2) and
    v_exp_f32 (T transcendentals/s)."""
    import ctypes as C
    import torch
    from paper_2310_03121_amd.build import CEIL_LIB
    lib = C.CDLL(CEIL_LIB)
    lib.nnp_ceiling_launch.restype = C.c_int
    lib.nnp_ceiling_launch.argtypes = [C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_void_p]
    lib.nnp_ceiling_work.restype = C.c_double
    lib.nnp_ceiling_work.argtypes = [C.c_int, C.c_int, C.c_int]
    blocks = 256 * 8 // 4 * 2  # two workgroups of 4 waves per CU
    sink = torch.zeros(blocks, dtype=torch.float32, device="cuda")
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    out = {}
    for name, kind in CEILING_KINDS.items():
        iters = {0: 100, 1: 50, 2: 100000, 3: 40000}[kind]  # 5-20 ms per launch
        for _ in range(2):
            assert lib.nnp_ceiling_launch(kind, blocks, iters, C.c_void_p(sink.data_ptr()),
                                          stream) == 0
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            lib.nnp_ceiling_launch(kind, blocks, iters, C.c_void_p(sink.data_ptr()), stream)
        e1.record()
        torch.cuda.synchronize()
        sec = e0.elapsed_time(e1) / 5 * 1e-3
        out[name] = lib.nnp_ceiling_work(kind, blocks, iters) / sec / 1e12
    out["units"] = "TFLOP/s (exp2: T/s)"
    return out


def measured_peak(bound, prec, issue):
    """The ceiling measured on this device for the roofline's bound: the MFMA
    issue loop of the path's precision for `mfma`, the FP32 FMA loop for
    `alu`, a 1 GiB device copy for `hbm`."""
    import torch
    if bound == "mfma":
        key = "mfma_bf16" if prec == "bf16" else "mfma_fp32"
        return {"value": issue[key], "unit": "TFLOP/s", "what": f"{key} issue loop"}
    if bound == "alu":
        return {"value": issue["valu_fma_fp32"] / 2, "unit": "Tops/s",
                "what": "fp32 FMA issue loop (one operation per FMA)"}
    src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    val = 2 * src.numel() / 1e9 / (e0.elapsed_time(e1) / 10 * 1e-3)
    del src, dst
    torch.cuda.empty_cache()
    return {"value": val, "unit": "GB/s", "what": "1 GiB device copy"}


def serve_leg(srv, reqs, rate=None, id_base=0):
    """Drive the continuous-batching server with a request stream.

    rate=None: closed loop (everything submitted at t=0; gives the saturation
    rate).  Otherwise requests are released at their Poisson arrival times
    scaled to `rate` per second.  Latency = completion - scheduled arrival.
    Request k is submitted as id id_base + k (ids stay unique on a server
    that serves several legs)."""
    gaps = np.diff([0.0] + [r.t_arrive for r in reqs])
    base_rate = len(reqs) / reqs[-1].t_arrive
    arrive = np.zeros(len(reqs)) if rate is None else np.cumsum(gaps) * base_rate / rate
    nxt = 0
    lat = {}
    t0 = time.perf_counter()
    t_report = 10.0
    while len(lat) < len(reqs):
        now = time.perf_counter() - t0
        if now > t_report:  # a long leg still reports every 10 s
            progress(f"  {len(lat)} of {len(reqs)} requests done, {srv.active} on the server, "
                     f"{srv.pending} pending")
            t_report += 10.0
        while nxt < len(reqs) and arrive[nxt] <= now:
            r = reqs[nxt]
            code = srv.submit(id_base + nxt, r.system.pos.astype(np.float64), r.vel,
                              r.system.species, r.n_steps)
            assert code == 0, code
            nxt += 1
        if srv.active == 0 and srv.pending == 0:
            if nxt < len(reqs):
                time.sleep(max(0.0, min(1e-3, arrive[nxt] - now)))
            continue
        srv.step()
        for rid in srv.poll():
            i = rid - id_base
            srv.result(rid, reqs[i].system.n_atoms)
            lat[i] = time.perf_counter() - t0 - arrive[i]
    wall = time.perf_counter() - t0
    atom_evals = sum(r.system.n_atoms * (r.n_steps + 1) for r in reqs)
    L = np.array(sorted(lat.values())) * 1e3
    return {"requests": len(reqs), "wall_s": wall, "req_per_s": len(reqs) / wall,
            "atoms_evals_per_s": atom_evals / wall, "p50_ms": float(np.percentile(L, 50)),
            "p99_ms": float(np.percentile(L, 99)), "server": srv.stats()}


def serving(at, mt, n_req=2000, n_warm=200, n_steps=100):
    import workloads as w
    from paper_2310_03121_amd import Potential
    allr = w.poisson_requests(n_warm + n_req, rate=1.0, seed=3, arrival_seed=30, n_steps=n_steps)
    warm, reqs = allr[:n_warm], allr[n_warm:]
    t_first = reqs[0].t_arrive
    for r in reqs:  # the timed stream's arrival times start from its first request
        r.t_arrive -= t_first
    out = {"workload": f"{n_req} MD requests after {n_warm} warm-up requests, 10-150 atoms "
                       f"(log-uniform), {n_steps} velocity-Verlet steps of 0.5 fs each, Poisson "
                       f"arrivals, 7 elements; server capacity 8,192 atoms / 256 molecules"}
    from paper_2310_03121_amd import Server
    for prec in ("bf16", "fp32"):
        pot = Potential.from_tables(at, mt, precision=prec, max_neighbors=64)
        # one server for all legs: its step graph is captured during the
        # warm-up, not inside a timed leg
        srv = Server(pot, hbm_budget_bytes=16 << 30, max_atoms=8192, max_mols=256, dt_fs=0.5,
                     mass_amu=w.MASS_AMU)
        serve_leg(srv, warm, id_base=0)  # warm-up: graph capture, kernel attributes, pages
        progress(f"serving {prec}: saturation")
        sat = serve_leg(srv, reqs, id_base=1 << 20)
        mu = sat["req_per_s"]
        r = {"saturation": sat}
        for k, f in enumerate((0.5, 0.8)):
            progress(f"serving {prec}: open loop at {f} of saturation")
            r[f"open_loop_{f}mu"] = serve_leg(srv, reqs, rate=f * mu, id_base=(k + 2) << 20)
        out[prec] = r
        del srv
        if prec == "bf16":
            # admission by an HBM budget: a server asked for 262,144 atoms
            # under a 1 GiB budget holds what fits, and the closed-loop stream
            # (about 104k atoms in all) waits for room
            srv = Server(pot, hbm_budget_bytes=1 << 30, max_atoms=262144, max_mols=4096,
                         dt_fs=0.5, mass_amu=w.MASS_AMU)
            serve_leg(srv, warm, id_base=0)
            progress("serving bf16: 1 GiB budget")
            out["bf16_budget_1GiB"] = {"saturation": serve_leg(srv, reqs, id_base=1 << 20)}
            del srv
        del pot
    return out


def cpu_baseline(s, S, budget_s=12.0, gpu=None, one_thread=False):
    """The FP64 oracle on a bounded sample of the workload (host cores).  The
    last oracle evaluation of the sample also gives the force and energy
    error of each GPU path (``gpu``: {precision: (E, F)} of the whole
    workload; the sample is its first molecules, which interact with nothing
    else, or the whole system).  one_thread: BLAS limited to one thread."""
    if one_thread:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):
            return cpu_baseline(s, S, budget_s, gpu, one_thread=False)
    import oracle
    import workloads as w
    try:
        from threadpoolctl import threadpool_info
        blas = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:
        blas = 1
    at, mt = w.aev_table(S), w.mlp_table(S)
    if s.box is None and s.n_mol > 1:
        k = min(s.n_mol, 64)
        sub = w.System(s.pos[: s.mol_offsets[k]], s.species[: s.mol_offsets[k]],
                       s.mol_offsets[: k + 1].copy(), None, S)
        desc = f"first {k} of {s.n_mol} molecules ({sub.n_atoms} atoms)"
    else:
        sub = s
        desc = f"whole system ({s.n_atoms} atoms)"
    n = 0
    t0 = time.perf_counter()
    while True:
        ref = oracle.energy_forces(sub, aev_table=at, mlp_table=mt)
        n += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    out = {"value": sub.n_atoms * n / dt, "unit": "atoms·evals/s", "cores": int(blas),
           "kind": "oracle",
           "sample": f"{desc}, {n} FP64 E+F evaluations in {dt:.1f} s; NumPy BLAS threads "
                     f"{blas}, elementwise work single-threaded; host has {os.cpu_count()} CPUs"}
    errors = {}
    for prec, (E, F) in (gpu or {}).items():
        Fs = F[: sub.n_atoms]
        errors[prec] = {
            "force_rmse_eV_per_A": float(np.sqrt(np.mean((Fs - ref.F) ** 2))),
            "force_rel_rms": float(np.linalg.norm(Fs - ref.F) / np.linalg.norm(ref.F)),
            "energy_max_abs_err_eV": float(np.max(np.abs(E[: sub.n_mol] - ref.E))),
            "force_error_sample": desc}
    return out, errors


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="batch")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-oracle", action="store_true",
                    help="accepted for older command lines; the force error is measured in the "
                         "CPU baseline leg (off with --no-cpu)")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving leg")
    ap.add_argument("--copy-probe", action="store_true",
                    help="first run a plain 512 MiB device copy (a known-size reference for "
                         "hardware byte counters)")
    ap.add_argument("--precision", default="both", choices=("both", "bf16", "fp32"))
    ap.add_argument("--nve", type=int, default=None,
                    help="NVE steps of the drift leg (default 1000 for water7667, else off)")
    ap.add_argument("--nve-dt", type=float, default=0.5, help="time step of the drift leg, fs")
    ap.add_argument("--nve-scale", type=float, default=0.05,
                    help="output-layer scale of the networks of the drift leg (random networks "
                         "at full scale heat the water box: kinetic energy x3.4 over 500 fs "
                         "at 0.1, x1.4 at 0.05)")
    ap.add_argument("--nve-relax", type=int, default=0,
                    help="FIRE iterations before the drift leg's velocities are drawn")
    ap.add_argument("--max-neighbors", type=int, default=None,
                    help="neighbor-list capacity of the handles (default per workload)")
    ap.add_argument("--ensemble", type=int, default=0,
                    help="also time an ensemble of this many networks (BF16 and FP32)")
    ap.add_argument("--ceilings", action="store_true",
                    help="also measure copy bandwidth and library GEMM rates on this device")
    args = ap.parse_args()
    if args.max_neighbors is not None:
        MAX_NEIGHBORS[args.workload] = args.max_neighbors
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the path is measured on one GPU's share "
              "(multi-GPU sharding is a design note, not implemented)", file=sys.stderr)
        raise SystemExit(2)

    import torch
    import workloads as w
    from paper_2310_03121_amd import Potential

    if args.copy_probe:
        src = torch.empty(512 << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    s, S, desc = workload(args.workload)
    at, mt = w.aev_table(S), w.mlp_table(S)
    dev = torch.device("cuda:0")
    pos = torch.from_numpy(s.pos).to(dev)
    sp = torch.from_numpy(s.species).to(dev)
    off = torch.from_numpy(s.mol_offsets).to(dev)
    box = s.box

    results = {}
    forces = {}  # last forces of each path: the CPU baseline leg measures their error
    precs = ("bf16", "fp32") if args.precision == "both" else (args.precision,)
    for prec in precs:
        pot = Potential.from_tables(at, mt, precision=prec,
                                    max_neighbors=MAX_NEIGHBORS[args.workload])
        progress(f"{prec}: timing {args.steps} evaluations")
        dt_eager, dt_graph, (E, F), stages = time_path(pot, pos, sp, off, box, args.steps,
                                                       args.warmup)
        dt = min(dt_eager, dt_graph)
        r = {"value": s.n_atoms * args.steps / dt, "ms_per_step": 1e3 * dt / args.steps,
             "launch": "graph replay" if dt_graph <= dt_eager else "eager",
             "eager_ms_per_step": 1e3 * dt_eager / args.steps,
             "graph_ms_per_step": 1e3 * dt_graph / args.steps,
             "stages_ms": {k: v[0] / max(v[1], 1) for k, v in stages.items() if v[1]}}
        forces[prec] = (E.cpu().numpy(), F.cpu().numpy().astype(np.float64))
        if prec == precs[0]:
            r["pairs"], r["triples"] = pair_counts(pot, s.n_atoms)
        if args.workload == "batch":
            progress(f"{prec}: nnp_backward leg")
            r["backward"] = backward_leg(pot, pos, sp, off, box, max(args.steps // 5, 3),
                                         max(args.warmup // 5, 2), mt)
            bw = r["backward"]
            if bw["weight_grad_tflops"] is not None:
                bw["weight_grad_frac_of_peak"] = bw["weight_grad_tflops"] / PEAK_TFLOPS[prec]
        if args.workload == "mol24":
            progress(f"{prec}: latency leg")
            r["latency"] = latency_leg(pot, pos, sp, off, box)
        n_nve = args.nve if args.nve is not None else (1000 if args.workload == "water7667" else 0)
        if n_nve:
            if args.nve_scale != 1.0:
                # the same networks with the output layer scaled: a gentler
                # random potential for the energy-conservation leg
                nve_pot = Potential.from_tables(at, mt.scaled_output(args.nve_scale),
                                                precision=prec,
                                                max_neighbors=MAX_NEIGHBORS[args.workload])
            else:
                nve_pot = pot
            progress(f"{prec}: NVE leg, {n_nve} steps")
            r["nve"] = nve_leg(nve_pot, s, n_steps=n_nve, dt=args.nve_dt,
                               relax_iters=args.nve_relax)
            r["nve"]["output_scale"] = args.nve_scale
            del nve_pot
        results[prec] = r
        del pot
        torch.cuda.empty_cache()

    main_prec = precs[0]
    main_r = results[main_prec]
    # roofline of the dominant kernel (largest per-launch device time)
    F_feat = mt.widths[0]
    sf = stage_flops(mt.widths, F_feat)
    st = main_r["stages_ms"]
    dom = max(st, key=st.get)
    traffic = profiled_traffic(dom, WORKLOAD_KEYS[args.workload] + "_" + main_prec)
    if dom in sf:
        achieved = sf[dom] * s.n_atoms / (st[dom] * 1e-3) / 1e12
        roof = {"kernel": dom, "bound": "mfma", "achieved": achieved, "peak": PEAK_TFLOPS[main_prec],
                "unit": "TFLOP/s", "frac": achieved / PEAK_TFLOPS[main_prec], "traffic": traffic,
                "flop_per_launch": sf[dom] * s.n_atoms, "avg_launch_ms": st[dom]}
    elif dom in AEV_OPS:
        op_pair, op_trip = AEV_OPS[dom]
        ops = op_pair * main_r["pairs"] + op_trip * main_r["triples"]
        achieved = ops / (st[dom] * 1e-3) / 1e12
        roof = {"kernel": dom, "bound": "alu", "achieved": achieved, "peak": PEAK_VALU_TOPS,
                "unit": "Tops/s (FP32 lane operations)", "frac": achieved / PEAK_VALU_TOPS,
                "traffic": traffic,
                "flop_per_launch": ops, "avg_launch_ms": st[dom],
                "pairs": main_r["pairs"], "triples": main_r["triples"]}
        pv = profiled_valu(dom, WORKLOAD_KEYS[args.workload] + "_" + main_prec)
        if pv is not None:
            # issue-slot use: a wave64 FP32 VALU instruction occupies a
            # SIMD for 2 cycles (32 lanes per clock); 1024 SIMDs at 2.4 GHz
            per_wave, waves = pv
            roof["valu_instr_per_wave"] = per_wave
            roof["valu_issue_frac"] = per_wave * waves * 2 / (1024 * 2.4e9 * st[dom] * 1e-3)
    else:
        roof = {"kernel": dom, "bound": "hbm", "achieved": None, "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "frac": None, "traffic": traffic, "avg_launch_ms": st[dom]}
    # the same kernel's mean duration in the committed kernel trace (event
    # timing adds the record/launch gap of one stage)
    roof["profiled_avg_ms"] = profiled_kernel_ms(dom, WORKLOAD_KEYS[args.workload] + "_" +
                                                 main_prec)
    # the same achieved rate against the ceiling measured here
    progress("issue-loop ceilings")
    issue = issue_ceilings()
    mp = measured_peak(roof["bound"], main_prec, issue)
    roof["measured_peak"] = mp
    roof["frac_of_measured"] = (roof["achieved"] / mp["value"]
                                if mp and roof.get("achieved") is not None else None)
    fwd, bwd = mlp_flops_per_atom(mt.widths, F_feat)
    path_tflops = (fwd + bwd) * s.n_atoms / (main_r["ms_per_step"] * 1e-3) / 1e12

    out = {
        "metric": METRIC,
        "value": main_r["value"],
        "unit": "atoms·evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_r["ms_per_step"],
        "launch": main_r["launch"],
        "eager_ms_per_step": main_r["eager_ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": main_prec,
        "data": "synthetic (seeded geometries and Gaussian weights)",
        "config": {"workload": desc, "n_atoms": s.n_atoms, "n_mol": s.n_mol,
                   "max_neighbors": MAX_NEIGHBORS[args.workload],
                   "mlp_widths": list(mt.widths), "precision_main": f"{main_prec} MLP, fp32 AEV/forces"},
        "force_rmse_eV_per_A": None,
        "force_rel_rms": None,
        "fp32_path": results.get("fp32"),
        "stages_ms": main_r["stages_ms"],
        "mlp_path_tflops": path_tflops,
        "mlp_path_frac_of_peak": path_tflops / PEAK_TFLOPS[main_prec],
        "roofline": roof,
        "measured_ceilings": issue,
    }
    for k in ("latency", "nve", "backward"):
        if k in main_r:
            out[k] = main_r[k]
    if not args.no_serve:
        progress("serving legs")
        sv = serving(w.aev_table(7), w.mlp_table(7))
        out["serving"] = sv
        out["p99_latency_ms_bf16_0.8mu"] = sv["bf16"]["open_loop_0.8mu"]["p99_ms"]
    if args.ensemble > 1:
        progress("ensemble leg")
        out["ensemble"] = ensemble_leg(s, at, S, args, results)
    if args.ceilings:
        out["ceilings"] = ceilings()
    if not args.no_cpu:
        # the oracle runs only here: the CPU baseline, whose last evaluation
        # of its sample also gives each path's force error
        progress("CPU baseline (oracle)")
        out["cpu_baseline"], errs = cpu_baseline(s, S, gpu=forces)
        for prec, e in errs.items():
            target = out if prec == main_prec else out.get("fp32_path")
            if target is not None:
                target.update(e)
        # the same oracle with BLAS on one thread (shorter sample)
        out["cpu_baseline_one_thread"], _ = cpu_baseline(s, S, budget_s=6.0, one_thread=True)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
