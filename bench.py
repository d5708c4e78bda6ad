"""Throughput of the fused collide-stream step on one MI355X.

Workload (default): the chemotaxis-fluid plume, 512 x 256 nodes, m = 2
(bacteria n, oxygen c) on D2Q5 + the D2Q9 fluid, step cut-off r(c), oxygen
consumption source, buoyancy, free-slip/Dirichlet top, no-slip/no-flux
bottom, periodic sides; populations stored as FP32 deviations and collided in
FP32.  One step = one lattice update of every node (the full fused update);
the FP64 steady-state residual is evaluated every 1000 steps inside the timed
region, as a steady solve does.  Inputs are resident in HBM before timing.

Prints one JSON line (rank 0).  Extra objects: ``roofline`` (algorithmic bytes
of the step kernel / its mean duration, against the HBM peak), ``cpu_baseline``
(the CPU oracle on a bounded sample of the same workload), ``fp64`` (same
workload with FP64 storage) and ``hbm_sweep`` (a periodic grid large enough to
leave the caches, where the HBM fraction is meaningful).
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

HBM_PEAK_GBS = 8000.0
METRIC = "MLUPS (fluid+m scalars) & HBM GB/s vs peak; wall time to steady: warm vs cold"


def bytes_per_lu(m: int, storage: str, n_src: int) -> int:
    """Algorithmic HBM bytes per lattice update: every population read once and
    written once, plus the previous-step source read and written."""
    b = {"f64": 8, "f32": 4, "f16": 2}[storage]
    a = 8 if storage == "f64" else 4
    return 2 * (9 + 5 * m) * b + 2 * n_src * a


def time_steps(solver, steps, warmup, residual_every=1000):
    import torch

    from paper_2101_03055_amd import lb

    stream = solver.stream
    solver.step(warmup)
    solver.residual()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    done = 0
    n_res = 0
    t0 = time.perf_counter()
    e0.record(stream)
    while done < steps:
        k = min(residual_every, steps - done)
        solver.step(k)
        done += k
        if done % residual_every == 0:
            lb.lb_residual(solver.handle, solver.m)  # synchronises (FP64 two-pass reduction)
            n_res += 1
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / 1e3, wall, n_res


def kernel_time(solver, launches):
    """Mean duration of one step launch, HIP events on the solver's stream,
    back-to-back launches (no host synchronisation in between)."""
    import torch

    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(solver.stream)
    solver.step(launches)
    e1.record(solver.stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3 / launches


def cpu_baseline(wl, phi0, u0, p0, budget_s=12.0):
    from oracle import oracle as O

    o = O.Oracle(wl, phi0, u0, p0)
    t0 = time.perf_counter()
    o.step(2)
    dt = max(time.perf_counter() - t0, 1e-6) / 2
    steps = max(2, int(budget_s / dt))
    t0 = time.perf_counter()
    o.step(steps)
    el = time.perf_counter() - t0
    lu = wl["nx"] * wl["ny"] * steps
    return {"value": lu / el / 1e6, "unit": "MLUPS", "cores": O.threads(), "kind": "oracle",
            "sample": f"{wl['name']}, FP64 oracle, {steps} steps from the same initial state ({el:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--mode", choices=["bench", "pmc", "copy"], default="bench",
                    help="pmc: only the timed workload's step kernel (for counter runs); "
                         "copy: a plain 1 GiB device copy to calibrate the byte counters")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the design notes describe how the domain would be sharded).", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2101_03055_amd import lb, workloads as W

    torch.cuda.set_device(0)
    if args.mode == "copy":
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")  # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": src.numel() * 4, "copies": 5}), flush=True)
        return
    wl, phi0, u0, p0 = W.chemotaxis_plume()
    if args.mode == "pmc":
        solver = lb.Solver(wl, phi0, u0, p0, storage="f32", phi_ref=[1.0, 1.0])
        solver.step(200)
        torch.cuda.synchronize()
        print(json.dumps({"pmc_steps": 200, "bytes_per_launch": bytes_per_lu(2, "f32", 1) * wl["nx"] * wl["ny"]}),
              flush=True)
        return
    N = wl["nx"] * wl["ny"]
    solver = lb.Solver(wl, phi0, u0, p0, storage="f32", phi_ref=[1.0, 1.0])
    n_src = 1
    el, wall, n_res = time_steps(solver, args.steps, args.warmup)
    mlups = N * args.steps / el / 1e6
    kt = kernel_time(solver, 1000)
    bpl = bytes_per_lu(2, "f32", n_src)
    achieved = bpl * N / kt / 1e9
    out = {
        "metric": METRIC, "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded PCG64 noise on n0, paper's plume parameters)",
        "config": {"workload": wl["name"], "nx": wl["nx"], "ny": wl["ny"], "m": 2,
                   "storage": "f32 deviations from phi_ref = (1, 1), rho0", "collision": "bgk",
                   "residual_every": 1000, "residual_evals_timed": n_res},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "k_step (even/odd AA launches alternate)",
                     "bytes_per_launch": bpl * N, "mean_launch_us": kt * 1e6,
                     "note": "working set 21 MB: resident in the 256 MB MALL, so achieved may exceed what HBM alone would give"},
    }
    if not args.no_extra:
        s64 = lb.Solver(wl, phi0, u0, p0, storage="f64")
        el64, _, _ = time_steps(s64, 2000, 100)
        kt64 = kernel_time(s64, 500)
        out["fp64"] = {"value": round(N * 2000 / el64 / 1e6, 1), "unit": "MLUPS",
                       "mean_launch_us": kt64 * 1e6,
                       "achieved_GBs": round(bytes_per_lu(2, "f64", 1) * N / kt64 / 1e9, 1)}
        del s64
        sweep = {}
        for storage, n in (("f64", 4096), ("f32", 4096)):
            wlb, pb, ub, ppb = W.taylor_green_blobs(n=n, steps=0)
            sb = lb.Solver(wlb, pb, ub, ppb, storage=storage, phi_ref=[1.0, 1.0])
            sb.step(20)
            ktb = kernel_time(sb, 100)
            bb = bytes_per_lu(2, storage, 0)
            ach = bb * n * n / ktb / 1e9
            sweep[f"{storage}_{n}x{n}"] = {"MLUPS": round(n * n / ktb / 1e6, 1), "achieved_GBs": round(ach, 1),
                                           "frac": round(ach / HBM_PEAK_GBS, 4), "mean_launch_us": ktb * 1e6,
                                           "bytes_per_lu": bb}
            del sb
            torch.cuda.empty_cache()
        out["hbm_sweep"] = sweep
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(wl, phi0, u0, p0)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
