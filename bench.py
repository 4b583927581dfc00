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


def mlp_flops_per_atom(widths, F):
    w = list(widths)
    w[0] = F
    fwd = sum(2 * w[l] * w[l + 1] for l in range(len(w) - 1))
    bwd = sum(2 * w[l] * w[l + 1] for l in range(len(w) - 2))  # input-gradient chain
    return fwd, bwd


def stage_flops(widths, F):
    """Algorithmic FLOPs per atom of each network stage."""
    w1, w2, w3 = widths[1], widths[2], widths[3]
    return {
        "mlp_layer1": 2 * F * w1, "mlp_layer2": 2 * w1 * w2, "mlp_layer3_head": 2 * w2 * w3 + 2 * w3,
        "mlp_bwd_layer3": 2 * w3 * w2, "mlp_bwd_layer2": 2 * w2 * w1, "mlp_bwd_dEdG": 2 * w1 * F,
    }


def workload(name):
    import workloads as w
    if name == "batch":
        return w.config_system(1), 7, "512 conformations x 64 atoms, 7 elements, 1008 features, no box"
    if name == "water1500":
        return w.config_system(2), 4, "1,500-water box (4,500 atoms), L=35.5 A, 4 elements, 384 features"
    if name == "water7667":
        return w.config_system(4), 7, "7,667-water box (23,001 atoms), L=61.2 A, 7 elements, 1008 features"
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
    # per-stage device times with HIP events on the launch stream, same steps
    pot.profile(True)
    for _ in range(steps):
        pot.energy_forces(pos, sp, off, box, out=out)
        pot.profile_collect()
    stages = pot.profile_read()
    pot.profile(False)
    return dt, out, stages


def cpu_baseline(s, S, budget_s=12.0):
    """The FP64 oracle on a bounded sample of the workload (host cores)."""
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
        oracle.energy_forces(sub, aev_table=at, mlp_table=mt)
        n += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": sub.n_atoms * n / dt, "unit": "atoms·evals/s", "cores": int(blas),
            "kind": "oracle",
            "sample": f"{desc}, {n} FP64 E+F evaluations in {dt:.1f} s; NumPy BLAS threads "
                      f"{blas}, elementwise work single-threaded; host has {os.cpu_count()} CPUs"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="batch")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-oracle", action="store_true", help="skip the force-error check")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the path is measured on one GPU's share "
              "(multi-GPU sharding is a design note, not implemented)", file=sys.stderr)
        raise SystemExit(2)

    import torch
    import oracle
    import workloads as w
    from paper_2310_03121_amd import Potential

    s, S, desc = workload(args.workload)
    at, mt = w.aev_table(S), w.mlp_table(S)
    dev = torch.device("cuda:0")
    pos = torch.from_numpy(s.pos).to(dev)
    sp = torch.from_numpy(s.species).to(dev)
    off = torch.from_numpy(s.mol_offsets).to(dev)
    box = s.box
    ref = None if args.no_oracle else oracle.energy_forces(s, aev_table=at, mlp_table=mt)

    results = {}
    for prec in ("bf16", "fp32"):
        pot = Potential.from_tables(at, mt, precision=prec)
        dt, (E, F), stages = time_path(pot, pos, sp, off, box, args.steps, args.warmup)
        r = {"value": s.n_atoms * args.steps / dt, "ms_per_step": 1e3 * dt / args.steps,
             "stages_ms": {k: v[0] / max(v[1], 1) for k, v in stages.items() if v[1]}}
        if ref is not None:
            Fn = F.cpu().numpy().astype(np.float64)
            r["force_rmse_eV_per_A"] = float(np.sqrt(np.mean((Fn - ref.F) ** 2)))
            r["force_rel_rms"] = float(np.linalg.norm(Fn - ref.F) / np.linalg.norm(ref.F))
            r["energy_max_abs_err_eV"] = float(np.max(np.abs(E.cpu().numpy() - ref.E)))
        results[prec] = r
        del pot
        torch.cuda.empty_cache()

    main_r = results["bf16"]
    # roofline of the dominant kernel (largest per-launch device time)
    F_feat = mt.widths[0]
    sf = stage_flops(mt.widths, F_feat)
    st = main_r["stages_ms"]
    dom = max(st, key=st.get)
    if dom in sf:
        achieved = sf[dom] * s.n_atoms / (st[dom] * 1e-3) / 1e12
        roof = {"kernel": dom, "bound": "mfma", "achieved": achieved, "peak": PEAK_TFLOPS["bf16"],
                "unit": "TFLOP/s", "frac": achieved / PEAK_TFLOPS["bf16"], "traffic": None,
                "flop_per_launch": sf[dom] * s.n_atoms, "avg_launch_ms": st[dom]}
    else:
        roof = {"kernel": dom, "bound": "alu", "achieved": None, "peak": None, "unit": None,
                "frac": None, "traffic": None, "avg_launch_ms": st[dom]}
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
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic (seeded geometries and Gaussian weights)",
        "config": {"workload": desc, "n_atoms": s.n_atoms, "n_mol": s.n_mol,
                   "mlp_widths": list(mt.widths), "precision_main": "bf16 MLP, fp32 AEV/forces"},
        "force_rmse_eV_per_A": main_r.get("force_rmse_eV_per_A"),
        "force_rel_rms": main_r.get("force_rel_rms"),
        "fp32_path": results["fp32"],
        "bf16_stages_ms": main_r["stages_ms"],
        "mlp_path_tflops": path_tflops,
        "mlp_path_frac_of_bf16_peak": path_tflops / PEAK_TFLOPS["bf16"],
        "roofline": roof,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(s, S)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
