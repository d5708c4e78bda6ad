"""Reduced-precision cascades for steady solves of the batched 128^2
double-diffusive cavities (the surrogate's held-out set), all warm-started
from the CNN surrogate's prediction and run to residual 1e-8 in FP64:

  fp64          the whole solve in FP64 storage;
  fp32>fp64     FP32 deviations to 1e-5, populations copied into FP64;
  fp16>fp64     FP16 deviations (x scale, stochastic rounding) to 1e-3, FP64
                restarted at equilibrium of the destaggered fields;
  fp16>fp32>fp64  FP16 to 1e-3, FP32 restarted at equilibrium of the
                destaggered fields to 1e-5, populations copied into FP64;
  'r' after a phase: hand over by a restart at equilibrium of the
                destaggered fields instead of a population copy; ':N' caps a
                phase at N steps (the batch's wall time is set by its slowest
                cavity, and a few cavities reach 1e-3 in FP16 much later
                than the rest);

plus the cold FP32>FP64 path (from rest) and the plain method (FP64, one
cavity at a time, from rest) on a subset.  The 128^2 batch of 185 cavities
holds 3.0 M nodes: 460 MB of FP64 populations (beyond the 256 MB MALL),
230 MB in FP32, 115 MB in FP16, so narrower storage moves fewer HBM bytes per
step.  Each path's wall time includes every phase and copy; accuracy is the
relative L2 distance of (u, v, T, C) to the plain FP64 solution on the
subset and to the all-FP64 batched solution on every cavity.

``python -m paper_2101_03055_amd.cascade_study --out FILE`` writes the
results as JSON.
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np

from . import lb, sg, workloads as W
from .run import destagger
from .surrogate_study import U_LAT, _sync, fields_of, plain_solve, predict, rel_l2, run_batch

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "data", "surrogate_ddc128.npz")
STUDY = os.path.join(HERE, "data", "surrogate_ddc128_study.json")
F16_SCALE, F16_SCALE_H = 1e3, 1e4  # scalar / fluid deviations are O(0.1) / O(0.01)


def _restart(batch, cases, status):
    """Cases restarted at equilibrium of the batch's destaggered fields (a
    cavity that diverged keeps its own initial fields)."""
    out = []
    for i, c in enumerate(cases):
        if status[i] == lb.LBB_DIVERGED:
            out.append(c)
        else:
            phi, u, p = batch.moments(i)
            out.append((c[0], phi, destagger(c[0], u), p))
    return out


def phases_of(path):
    """'fp16:40000>fp32r>fp64' -> [(storage, step cap or None, restart)]: a phase
    name ending in 'r' hands its fields over by a restart at equilibrium of the
    destaggered fields instead of copying populations (FP16 phases always
    restart); ':N' caps the phase at N steps."""
    out = []
    for ph in path.split(">"):
        name, _, cap = ph.partition(":")
        restart = name.endswith("r") or name.startswith("fp16")
        out.append((name.rstrip("r"), int(cap) if cap else None, restart))
    return out


def solve(cases, path, tol=1e-8, tol32=1e-5, tol16=1e-3, max_steps=3_000_000, log=print):
    """One cascade over the whole batch; returns (record, fields)."""
    quiet = lambda s: None
    tols = {"fp16": tol16, "fp32": tol32, "fp64": tol}
    _sync()
    t0 = time.perf_counter()
    phases = {}
    cur = cases
    prev = None  # (batch, status, restart) of the previous phase
    for storage, cap, restart in phases_of(path):
        if prev is not None and prev[2]:
            cur = _restart(prev[0], cur, prev[1])
            prev[0].close()
            prev = None
        kw = {"fp16_scale": F16_SCALE, "fp16_scale_h": F16_SCALE_H} if storage == "fp16" else {}
        b = lb.Batch(cur, storage=storage[2:] and "f" + storage[2:], phi_ref=None if storage == "fp64" else [0.5, 0.5],
                     **kw)
        if prev is not None:   # copy populations from the previous (FP32) phase
            for i in range(len(cases)):
                if prev[1][i] != lb.LBB_DIVERGED:
                    lb.lbb_copy_cavity(b.handle, i, prev[0].handle, i)
            prev[0].close()
        s, st, secs = run_batch(b, tols[storage], 1000, cap or max_steps, window=min(50000, cap or 50000), log=quiet)
        phases[storage] = {"steps_median": float(np.median(s)), "seconds": secs,
                           "cap": cap, "reached_tol": int(np.sum(np.asarray(st) == lb.LBB_CONVERGED))}
        prev = (b, st, restart)
    b64 = prev[0]
    _sync()
    total = time.perf_counter() - t0
    fields = [fields_of(b64, i) for i in range(len(cases))]
    st = prev[1]
    rec = {"path": path, "seconds": total, "phases": phases,
           "converged": int(np.sum(np.asarray(st) == lb.LBB_CONVERGED)), "cavities": len(cases)}
    b64.close()
    log(f"  {path}: {total:.1f} s, converged {rec['converged']}/{len(cases)}, "
        + ", ".join(f"{k} {v['steps_median']:.0f} steps {v['seconds']:.1f} s" for k, v in phases.items()))
    return rec, fields


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--out", default=None)
    ap.add_argument("--cases", type=int, default=0, help="first n steady held-out cavities (0: all)")
    ap.add_argument("--plain", type=int, default=8)
    args = ap.parse_args()
    log = lambda s: print(s, flush=True)
    with open(STUDY) as fh:
        study = json.load(fh)
    pc = study["batched"]["per_case"]
    steady = [i for i in range(len(pc["status_warm"])) if pc["status_warm"][i] == 1 or pc["status_cold"][i] == 1]
    if args.cases:
        steady = steady[: args.cases]
    seeds = [20000 + i for i in steady]
    pds = [W.sweep_case(s, 128) for s in seeds]
    cases = [W.ddc_case(pd) for pd in pds]
    params = np.array([W.normalise(pd) for pd in pds], dtype=np.float32)
    nodes = sum(c[0]["nx"] * c[0]["ny"] for c in cases)
    log(f"{len(cases)} steady held-out cavities, {nodes} nodes")
    net = sg.Surrogate(16, 128, 128)
    net.set_weights(np.load(WEIGHTS)["w"])
    _sync()
    t0 = time.perf_counter()
    pred = predict(net, params)
    t_pred = time.perf_counter() - t0
    warm_cases = [(wl, np.stack([f[2], f[3]]), np.stack([f[0], f[1]]) * U_LAT, None)
                  for (wl, _, _, _), f in zip(cases, pred)]
    out = {"cavities": len(cases), "nodes": nodes, "predict_seconds": t_pred, "tol": 1e-8, "tol32": 1e-5,
           "tol16": 1e-3, "fp16_scale": [F16_SCALE, F16_SCALE_H], "paths": {}}
    ref = None
    for path in ("fp64", "fp32>fp64", "fp32r>fp64", "fp16:40000>fp64", "fp16:40000>fp32>fp64"):
        rec, f = solve(warm_cases, path, log=log)
        rec["seconds_with_prediction"] = rec["seconds"] + t_pred
        if ref is None:
            ref = f
        rec["relL2_vs_fp64_batched_max"] = max(rel_l2(a, b) for a, b in zip(f, ref))
        out["paths"]["warm " + path] = rec
        out["paths"]["warm " + path]["fields"] = f  # kept for the plain comparison below
    rec, _ = solve(cases, "fp32>fp64", log=log)
    out["paths"]["cold fp32>fp64"] = rec
    plain = []
    for i in range(min(args.plain, len(cases))):
        steps, st, secs, f = plain_solve(cases[i])
        plain.append({"cavity": steady[i], "steps": steps, "status": st, "seconds": secs,
                      **{f"relL2 {k}": rel_l2(v["fields"][i], f) for k, v in out["paths"].items() if "fields" in v}})
        log(f"  plain cavity {steady[i]}: {steps} steps, {secs:.2f} s")
    for v in out["paths"].values():
        v.pop("fields", None)
    per_plain = float(np.mean([p["seconds"] for p in plain])) if plain else None
    out["plain"] = {"cavities": plain, "seconds_per_cavity": per_plain}
    for k, v in out["paths"].items():
        secs = v.get("seconds_with_prediction", v["seconds"])
        v["seconds_per_cavity"] = secs / len(cases)
        if per_plain:
            v["speedup_vs_plain"] = per_plain / v["seconds_per_cavity"]
        v["speedup_vs_warm_fp64"] = out["paths"]["warm fp64"]["seconds_with_prediction"] / secs
    log(json.dumps({k: {kk: vv for kk, vv in v.items() if kk != "phases"} for k, v in out["paths"].items()},
                   indent=1))
    if args.out:
        with open(args.out, "w") as fh:
            json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
