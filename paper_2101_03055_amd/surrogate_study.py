"""Surrogate warm start study: LB-generated training data, training on the
GPU with the library's own kernels, and steady solves warm vs cold.

Pipeline (all on one GPU):
 1. dataset: cavities drawn from the sweep law at L x L (one seed each) are
    solved to steady state by the batched FP32 solver (MRT fluid); targets
    are (u / u_lat, v / u_lat, T, C), inputs the normalised parameters;
 2. training: the CNN (sg.h) with Adam for a number of epochs (learning
    rate lowered 3x after 60 % and again after 85 % of them);
 3. evaluation on held-out seeds, every path to residual 1e-8:
    - plain   : FP64 single-domain solve from rest, one cavity after the other
                (the method as the paper runs it), on a subset;
    - cold    : batched FP32 phase (to its noise floor) + batched FP64 finish,
                from rest;
    - warm    : the same batched path started from the surrogate's prediction;
    errors are relative L2 against the plain FP64 solution (subset) and
    against the cold batched solution (all).

``python -m paper_2101_03055_amd.surrogate_study --out DIR`` writes
summary.json and the trained weights (weights.npz) to DIR.
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np

from . import lb, sg, workloads as W

U_LAT = 0.1


def _sync():
    import torch

    torch.cuda.synchronize()


def run_batch(batch, tol, check_every, max_steps, window=20000, label="", log=print):
    """lbb_run in windows (progress between windows); returns steps, status, seconds."""
    t0 = time.perf_counter()
    done = 0
    while done < max_steps:
        k = min(window, max_steps - done)
        steps, status, res = batch.run(tol=tol, check_every=check_every, max_steps=k)
        done += k
        left = int(np.sum(status == lb.LBB_RUNNING))
        log(f"  {label}: {done} steps, running {left}, converged {int(np.sum(status == lb.LBB_CONVERGED))}, "
            f"diverged {int(np.sum(status == lb.LBB_DIVERGED))}, {time.perf_counter() - t0:.1f}s")
        if left == 0:
            break
    return steps, status, time.perf_counter() - t0


def fields_of(batch, i):
    phi, u, _ = batch.moments(i)
    return np.stack([u[0] / U_LAT, u[1] / U_LAT, phi[0], phi[1]])


def generate(seeds, L, tol=5e-6, max_steps=600_000, check_every=1000, log=print):
    pds = [W.sweep_case(s, L) for s in seeds]
    cases = [W.ddc_case(pd) for pd in pds]
    t0 = time.perf_counter()
    b = lb.Batch(cases, storage="f32", phi_ref=[0.5, 0.5])
    tx, ty, us = b.autotune(10)
    log(f"  dataset batch of {len(seeds)}: tile {tx}x{ty}, {us:.1f} us/step")
    steps, status, secs = run_batch(b, tol, check_every, max_steps, window=50000, label="dataset", log=log)
    ok = np.where(status == lb.LBB_CONVERGED)[0]
    params = np.array([W.normalise(pds[i]) for i in ok], dtype=np.float32)
    fields = np.stack([fields_of(b, i) for i in ok]).astype(np.float32)
    info = {"cases": len(seeds), "converged": int(len(ok)), "diverged": int(np.sum(status == lb.LBB_DIVERGED)),
            "unsteady_or_slow": int(np.sum(status == lb.LBB_RUNNING)), "solve_seconds": secs,
            "total_seconds": time.perf_counter() - t0, "steps_median": float(np.median(steps)),
            "tile": [tx, ty]}
    b.close()
    return params, fields, [seeds[i] for i in ok], info


def train(params, fields, epochs, batch=16, lr=1e-3, seed=0, log=print):
    """Adam in three phases of decreasing learning rate (lr, lr/3, lr/10 over
    60 %, 25 % and 15 % of the epochs); the moment estimates restart with
    each phase."""
    import torch

    L = fields.shape[-1]
    dp = torch.tensor(params, device="cuda")
    df = torch.tensor(fields, device="cuda")
    losses = []
    t0 = time.perf_counter()
    bounds = [0, int(round(0.6 * epochs)), int(round(0.85 * epochs)), epochs]
    w = sg.init_weights(seed)
    net = None
    for ph, scale in enumerate((1.0, 1.0 / 3.0, 0.1)):
        e_begin, e_end = bounds[ph], bounds[ph + 1]
        if e_end <= e_begin:
            continue
        if net is not None:
            w = net.get_weights()
            net.close()
        net = sg.Surrogate(batch, fields.shape[-2], L, lr=lr * scale)
        net.set_weights(w)
        per = max(1, (e_end - e_begin) // 5)
        for e0 in range(e_begin, e_end, per):
            k = min(per, e_end - e0)
            losses += net.train_epochs(dp, df, len(params), k, seed=seed + e0).tolist()
            log(f"  train: epoch {e0 + k}/{epochs} (lr {lr * scale:.1e}), loss {losses[-1]:.3e}, "
                f"{time.perf_counter() - t0:.1f}s")
    return net, losses, time.perf_counter() - t0


def predict(net, params, smooth=True):
    """Surrogate fields [n][4][H][W], prepared for a warm start on the GPU:
    one [1 2 1] pass (grid-scale noise excites lattice modes that decay very
    slowly) and removal of the lattice-staggered velocity sums (they would
    persist as an undamped period-2 oscillation; sg_destagger).  smooth=False
    returns the raw network output."""
    import torch

    n = len(params)
    L = net.cfg.width
    out = torch.empty((n, 4, net.cfg.height, L), dtype=torch.float32, device="cuda")
    dp = torch.tensor(np.asarray(params, dtype=np.float32), device="cuda")
    net.predict(dp, n, out)
    if smooth:
        sm = torch.empty_like(out)
        sg.smooth(out, sm)
        sg.destagger(sm)
        out = sm
    _sync()
    return out.cpu().numpy().astype(np.float64)


def solve_path(cases, init_fields, tol32=1e-5, tol=1e-8, max_steps=1_500_000, label="", log=print):
    """Batched FP32 phase then batched FP64 finish; init_fields None = from rest.
    A warm-started cavity that diverges in the FP32 phase falls back to a cold
    start: its FP64 phase begins from rest instead of from the copied state
    (the LB iteration decides the prediction's error)."""
    cold_cases = cases
    if init_fields is not None:
        cases = [(wl, np.stack([f[2], f[3]]), np.stack([f[0], f[1]]) * U_LAT, None)
                 for (wl, _, _, _), f in zip(cases, init_fields)]
    _sync()
    t0 = time.perf_counter()
    b32 = lb.Batch(cases, storage="f32", phi_ref=[0.5, 0.5])
    s32, st32, _ = run_batch(b32, tol32, 1000, max_steps, window=50000, label=label + " fp32", log=log)
    fallback = [i for i in range(len(cases)) if init_fields is not None and st32[i] == lb.LBB_DIVERGED]
    if fallback:
        log(f"  {label}: {len(fallback)} warm start(s) diverged; restarting them from rest")
    b64 = lb.Batch([cold_cases[i] if i in fallback else cases[i] for i in range(len(cases))], storage="f64")
    for i in range(len(cases)):
        if i not in fallback:
            lb.lbb_copy_cavity(b64.handle, i, b32.handle, i)
    s64, st64, _ = run_batch(b64, tol, 1000, max_steps, window=50000, label=label + " fp64", log=log)
    _sync()
    secs = time.perf_counter() - t0
    fields = [fields_of(b64, i) for i in range(len(cases))]
    steps = [int(s64[i]) + (int(s32[i]) if i in fallback else 0) for i in range(len(cases))]
    return {"steps_fp32": s32.tolist(), "steps_total": steps, "status": st64.tolist(), "seconds": secs,
            "fallback": fallback}, fields


def plain_solve(case, tol=1e-8, max_steps=3_000_000):
    s = lb.Solver(*case, storage="f64")
    _sync()
    t0 = time.perf_counter()
    steps, res, st = s.solve_steady(tol, 1000, max_steps)
    _sync()
    secs = time.perf_counter() - t0
    phi, u, _ = s.moments()
    f = np.stack([u[0] / U_LAT, u[1] / U_LAT, phi[0], phi[1]])
    s.close()
    return steps, st, secs, f


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--L", type=int, default=128)
    ap.add_argument("--train", type=int, default=2000)
    ap.add_argument("--test", type=int, default=200)
    ap.add_argument("--plain", type=int, default=16, help="test cavities also solved by the plain FP64 method")
    ap.add_argument("--epochs", type=int, default=200)
    ap.add_argument("--tol32", type=float, default=1e-5, help="residual that ends the FP32 phase")
    ap.add_argument("--data-tol", type=float, default=5e-6)
    ap.add_argument("--weights", default=None, help="trained weights (.npz): skip dataset and training")
    args = ap.parse_args()
    os.makedirs(args.out, exist_ok=True)
    log = lambda s: print(s, flush=True)
    summary = {"L": args.L, "u_lat": U_LAT, "collision": "bgk", "storage": "f32 phase + f64 finish",
               "tol32": args.tol32, "tol": 1e-8}

    def save():
        with open(os.path.join(args.out, "summary.json"), "w") as fh:
            json.dump(summary, fh, indent=1)

    if args.weights:
        net = sg.Surrogate(16, args.L, args.L)
        net.set_weights(np.load(args.weights)["w"])
        summary["weights"] = os.path.basename(args.weights)
    else:
        log("dataset")
        params, fields, seeds, info = generate(list(range(10000, 10000 + args.train)), args.L, tol=args.data_tol,
                                               log=log)
        summary["dataset"] = info
        save()
        log("training")
        net, losses, tsecs = train(params, fields, args.epochs, log=log)
        summary["training"] = {"epochs": args.epochs, "samples": len(params), "seconds": tsecs,
                               "loss_first": losses[0], "loss_last": losses[-1]}
        np.savez(os.path.join(args.out, "weights.npz"), w=net.get_weights(), losses=np.array(losses))
        save()

    log("evaluation")
    tseeds = list(range(20000, 20000 + args.test))
    tpds = [W.sweep_case(s, args.L) for s in tseeds]
    cases = [W.ddc_case(pd) for pd in tpds]
    tparams = np.array([W.normalise(pd) for pd in tpds], dtype=np.float32)
    _sync()
    t0 = time.perf_counter()
    pred = predict(net, tparams)
    t_pred = time.perf_counter() - t0
    warm, f_warm = solve_path(cases, pred, tol32=args.tol32, label="warm", log=log)
    warm["seconds_predict"] = t_pred
    cold, f_cold = solve_path(cases, None, tol32=args.tol32, label="cold", log=log)
    ok = [i for i in range(len(cases)) if warm["status"][i] == 1 and cold["status"][i] == 1]
    summary["batched"] = {
        "cases": len(cases), "both_converged": len(ok),
        "warm_seconds": warm["seconds"] + t_pred, "cold_seconds": cold["seconds"],
        "speedup_warm_vs_cold": cold["seconds"] / (warm["seconds"] + t_pred),
        "steps_warm_median": float(np.median([warm["steps_total"][i] for i in ok])),
        "steps_cold_median": float(np.median([cold["steps_total"][i] for i in ok])),
        "prediction_relL2_vs_cold_median": float(np.median([rel_l2(pred[i], f_cold[i]) for i in ok])),
        "warm_relL2_vs_cold_max": max(rel_l2(f_warm[i], f_cold[i]) for i in ok),
        "warm_helps_fraction": float(np.mean([warm["steps_total"][i] < cold["steps_total"][i] for i in ok])),
        "steps_fp32_warm_median": float(np.median([warm["steps_fp32"][i] for i in ok])),
        "steps_fp32_cold_median": float(np.median([cold["steps_fp32"][i] for i in ok])),
        "per_case": {"steps_warm": warm["steps_total"], "steps_cold": cold["steps_total"],
                     "steps_fp32_warm": warm["steps_fp32"], "steps_fp32_cold": cold["steps_fp32"],
                     "status_warm": warm["status"], "status_cold": cold["status"]},
    }
    save()
    # time to steady: batch wall times are set by the slowest cavity, and
    # cavities that never become steady run to the step cap either way; time
    # both paths again on the cavities that became steady in either run
    steady = [i for i in range(len(cases)) if warm["status"][i] == 1 or cold["status"][i] == 1]
    log(f"time to steady: {len(steady)} cavities")
    _sync()
    t0 = time.perf_counter()
    pred_s = predict(net, tparams[steady])
    t_pred_s = time.perf_counter() - t0
    sub = [cases[i] for i in steady]
    warm_s, _ = solve_path(sub, pred_s, tol32=args.tol32, max_steps=3_000_000, label="warm (steady set)", log=log)
    cold_s, _ = solve_path(sub, None, tol32=args.tol32, max_steps=3_000_000, label="cold (steady set)", log=log)
    summary["time_to_steady"] = {
        "cavities": len(steady), "max_steps_per_phase": 3_000_000,
        "steady_warm": int(sum(1 for v in warm_s["status"] if v == 1)),
        "steady_cold": int(sum(1 for v in cold_s["status"] if v == 1)),
        "warm_seconds": warm_s["seconds"] + t_pred_s, "cold_seconds": cold_s["seconds"],
        "speedup_warm_vs_cold": cold_s["seconds"] / (warm_s["seconds"] + t_pred_s),
    }
    save()
    log("plain FP64 reference on a subset")
    plain = []
    for i in ok[: args.plain]:
        steps, st, secs, f = plain_solve(cases[i])
        plain.append({"case": i, "steps": steps, "status": st, "seconds": secs,
                      "warm_relL2": rel_l2(f_warm[i], f), "cold_relL2": rel_l2(f_cold[i], f),
                      "pred_relL2": rel_l2(pred[i], f)})
        log(f"  plain case {i}: {steps} steps {secs:.2f}s warm err {plain[-1]['warm_relL2']:.2e}")
    per_case_plain = float(np.mean([p["seconds"] for p in plain])) if plain else None
    summary["plain_subset"] = plain
    if plain:
        summary["speedup_vs_plain"] = {
            "plain_seconds_per_case": per_case_plain,
            "warm_batched_seconds_per_case": summary["batched"]["warm_seconds"] / len(cases),
            "speedup": per_case_plain / (summary["batched"]["warm_seconds"] / len(cases)),
            "warm_relL2_vs_plain_max": max(p["warm_relL2"] for p in plain),
        }
        tts = summary["time_to_steady"]
        tts["warm_seconds_per_cavity"] = tts["warm_seconds"] / tts["cavities"]
        tts["speedup_vs_plain"] = per_case_plain / tts["warm_seconds_per_cavity"]
    save()
    log(json.dumps({k: summary[k] for k in ("dataset", "training", "batched", "time_to_steady") if k in summary},
                   indent=1))


if __name__ == "__main__":
    main()
