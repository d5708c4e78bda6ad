"""Run a named workload configuration on the GPU.

    python -m paper_2101_03055_amd.run CONFIG [--storage f64|f32|f16] [--steps N] [--steady]
                                       [--out fields.npz]

CONFIG is a file name under ``configs/`` (without ``.json``) or a path.  A
transient run advances the configured number of steps (or ``--steps``) and
reports the step rate, the per-species masses and the fields; a steady run
(``--steady``, or a configuration whose run section sets ``tol``) iterates to
the configured residual.  With reduced-precision storage a steady run first
iterates in that storage to ``tol32`` (FP32, 1e-5 unless the configuration
sets it) or ``tol16`` (FP16, 1e-3): reduced-precision storage cannot resolve
residuals near 1e-8.  It then finishes in FP64 storage, from the copied FP32
populations, or from equilibrium of the FP16 fields with the lattice-staggered
velocity sums removed.  A sweep configuration runs as one
batch (reduced-precision phase, then FP64).  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from . import lb, workloads as W


def _sync():
    import torch

    torch.cuda.synchronize()


def _transient(case, storage, phi_ref, steps):
    wl = case[0]
    s = lb.Solver(*case, storage=storage, phi_ref=phi_ref)
    s.step(min(steps, 64))  # first launches and graph build outside the timed part
    _sync()
    t0 = time.perf_counter()
    s.step(steps - min(steps, 64))
    _sync()
    secs = time.perf_counter() - t0
    timed = steps - min(steps, 64)
    mass, _ = s.mass()
    phi, u, p = s.moments()
    out = {"steps": s.t, "seconds": secs,
           "MLUPS": wl["nx"] * wl["ny"] * timed / secs / 1e6 if timed and secs > 0 else None,
           "mass": mass.tolist()}
    s.close()
    return out, (phi, u, p)


def destagger(wl, u):
    """Removes the lattice-staggered velocity sums sum (-1)^x u_x and
    sum (-1)^y u_y.  With walls (or an even periodic extent) on an axis the
    collide-stream update maps Q = sum (-1)^x j_x to -(Q + sum (-1)^x F_x)
    exactly, an undamped period-2 mode whose fixed point is the state with no
    staggered velocity sum (where a start from rest sits); a state carried
    over from FP16 storage is generally off it, and no number of FP64 steps
    would remove the difference."""
    u = np.array(u, dtype=np.float64, copy=True)
    ny, nx = wl["ny"], wl["nx"]
    per_x = wl["fluid_bc"][0] == "periodic"
    per_y = wl["fluid_bc"][2] == "periodic"
    if not per_x or nx % 2 == 0:
        sx = np.where(np.arange(nx) % 2 == 0, 1.0, -1.0)[None, :]
        u[0] -= np.mean(u[0] * sx) * sx
    if not per_y or ny % 2 == 0:
        sy = np.where(np.arange(ny) % 2 == 0, 1.0, -1.0)[:, None]
        u[1] -= np.mean(u[1] * sy) * sy
    return u


def _steady(case, storage, phi_ref, tol, tol_reduced, check_every, max_steps):
    _sync()
    t0 = time.perf_counter()
    out = {}
    if storage == "f64":
        s = lb.Solver(*case, storage="f64")
        steps, res, st = s.solve_steady(tol, check_every, max_steps)
        out.update(steps=steps, status=int(st), residual=res.tolist())
    else:
        r = lb.Solver(*case, storage=storage, phi_ref=phi_ref)
        n_r, res_r, st_r = r.solve_steady(tol_reduced, check_every, max_steps)
        if st_r == lb.LB_ENONFINITE:  # the reduced-precision phase diverged: start over in FP64
            s = lb.Solver(*case, storage="f64")
        elif storage == "f32":  # FP32 values are exact in FP64: carry the populations over
            s = lb.Solver(*case, storage="f64")
            lb.lb_copy_state(s.handle, r.handle)
        else:  # FP16: restart FP64 at equilibrium of the fields, off the staggered mode
            phi, u, p = r.moments()
            s = lb.Solver(case[0], phi, destagger(case[0], u), p, storage="f64")
        r.close()
        steps, res, st = s.solve_steady(tol, check_every, max_steps)
        out.update(steps_reduced=n_r, status_reduced=int(st_r), steps_fp64=steps, status=int(st),
                   residual=res.tolist())
    _sync()
    out["seconds"] = time.perf_counter() - t0
    mass, _ = s.mass()
    out["mass"] = mass.tolist()
    fields = s.moments()
    s.close()
    return out, fields


def _sweep(cases, storage, phi_ref, tol, tol32, check_every, max_steps, keep_fields=False):
    from .surrogate_study import run_batch

    quiet = lambda s: None
    _sync()
    t0 = time.perf_counter()
    b = lb.Batch(cases, storage=storage, phi_ref=phi_ref)
    tile = b.autotune(10)[:2]
    if storage == "f32":  # FP32 values are exact in FP64: carry the populations over
        s_r, st_r, _ = run_batch(b, tol32, check_every, max_steps, window=50000, log=quiet)
        b64 = lb.Batch(cases, storage="f64")
        for i in range(len(cases)):
            if st_r[i] != lb.LBB_DIVERGED:
                lb.lbb_copy_cavity(b64.handle, i, b.handle, i)
        b.close()
        b = b64
    elif storage == "f16":  # restart FP64 at equilibrium of each cavity's fields, off the staggered mode
        s_r, st_r, _ = run_batch(b, tol32, check_every, max_steps, window=50000, log=quiet)
        restart = []
        for i, c in enumerate(cases):
            if st_r[i] == lb.LBB_DIVERGED:
                restart.append(c)
            else:
                phi, u, p = b.moments(i)
                restart.append((c[0], phi, destagger(c[0], u), p))
        b.close()
        b = lb.Batch(restart, storage="f64")
    s64, st64, _ = run_batch(b, tol, check_every, max_steps, window=50000, log=quiet)
    _sync()
    secs = time.perf_counter() - t0
    st64 = np.asarray(st64)
    out = {"cavities": len(cases), "tile": list(tile), "seconds": secs,
           "converged": int((st64 == lb.LBB_CONVERGED).sum()), "diverged": int((st64 == lb.LBB_DIVERGED).sum()),
           "steps_fp64_median": float(np.median(s64))}
    fields = [b.moments(i) for i in range(len(cases))] if keep_fields else None
    b.close()
    return out, fields


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("config")
    ap.add_argument("--storage", choices=["f64", "f32", "f16"], default=None)
    ap.add_argument("--steps", type=int, default=None, help="transient run of this many steps")
    ap.add_argument("--steady", action="store_true", help="iterate to the configured residual")
    ap.add_argument("--max-steps", type=int, default=None)
    ap.add_argument("--out", default=None, help="write phi, u, p to this .npz (single domains)")
    args = ap.parse_args(argv)

    cfg, cases = W.load_config(args.config)
    run = cfg.get("run", {})
    storage = args.storage or (run.get("storage") or ["f64"])[0]
    phi_ref = run.get("phi_ref")
    tol = run.get("tol", 1e-8)
    # residual that ends the reduced-precision phase: above each storage's noise
    # floor (FP32 ~3e-7, FP16 ~1e-4 on the double-diffusive cavity)
    tol_reduced = run.get("tol16", 1e-3) if storage == "f16" else run.get("tol32", 1e-5)
    check_every = run.get("check_every", 1000)
    max_steps = args.max_steps or run.get("max_steps", 5_000_000)
    if cfg["workload"] == "sweep_case":
        raise SystemExit("the surrogate configuration runs through `python -m paper_2101_03055_amd.surrogate_study`")
    rec = {"config": os.path.basename(args.config).removesuffix(".json"), "storage": storage}
    fields = None
    if cfg["workload"] == "sweep":
        rec.update(_sweep(cases, storage, phi_ref, tol, tol_reduced, check_every, max_steps)[0])
    elif args.steady or (args.steps is None and "tol" in run):
        out, fields = _steady(cases[0], storage, phi_ref, tol, tol_reduced, check_every, max_steps)
        rec.update(out)
    else:
        steps = args.steps if args.steps is not None else run.get("steps", 1000)
        steps = steps[0] if isinstance(steps, list) else steps
        out, fields = _transient(cases[0], storage, phi_ref, int(steps))
        rec.update(out)
    if args.out and fields is not None:
        phi, u, p = fields
        np.savez(args.out, phi=phi, u=u, p=p)
        rec["out"] = args.out
    print(json.dumps(rec), flush=True)
    return rec


if __name__ == "__main__":
    sys.exit(0 if main() else 1)
