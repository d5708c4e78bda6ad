"""Throughput of the fused collide-stream step on one MI355X.

Workload (headline): the batched parameter sweep of double-diffusive cavities
-- 256 cavities with Soret/Dufour cross-diffusion (m = 2: T and C on D2Q5 plus
the D2Q9 fluid), sides drawn from {64, 96, ..., 256}, Ra log-uniform in
[1e3, 1e6], Le U[1, 5], Nc U[-2, 2], Sr, Df U[0, 0.5], Pr 0.71 (seed 4): 8.0 M
nodes, a 608 MB FP32 state, well beyond the 256 MB MALL.  Populations are
stored as FP32 deviations and collided in FP32; one step = one launch over
the tile list of every cavity (autotuned tile shape).  Every full window of
1000 steps inside the timed region ends with the FP64 per-cavity residual of
a steady sweep.  Inputs are resident in HBM before timing.

Prints one JSON line.  Besides the contract's fields:
  roofline       algorithmic bytes of the batched step kernel per launch / its
                 mean duration (HIP events on the batch's stream, back-to-back
                 launches) against the HBM peak; `traffic` from rocprofv3
                 FETCH_SIZE/WRITE_SIZE (profiles/*.traffic.json) while the kernel
                 sources are unchanged, else null;
  cpu_baseline   the FP64 CPU oracle on a bounded sample of the same workload
                 (a stated subset of the cavities);
  production_run the same batch through lbb_run over 2000 steps: residual
                 windows of 1000 steps, snapshots included;
  plume          the chemotaxis-fluid plume, 512 x 256 (FP32 and FP64): a
                 21 MB state resident in the MALL (cache-resident rates);
  hbm_sweep      periodic 4096^2 grids (FP64/FP32/FP16 storage, BGK and MRT);
  steady_warm_vs_cold  double-diffusive cavities at 128^2 solved to residual
                 1e-8 (batched FP32 phase + FP64 finish) from rest and from the
                 CNN surrogate's prediction (weights from the surrogate study);
  surrogate      training / inference throughput of the CNN (BF16 MFMA);
  cde_sweep      the no-fluid model (prescribed velocity) on 4096^2;
  sweep_3d       the 3-D path (D3Q7 + D3Q19) on a periodic 256^3 box.
Long runs of 2-D steps are replayed by the library as HIP graphs of 64 launches.
Modes for profiling: --mode pmc | copy | sweep | batch | plume | surrogate | cde | 3d.
--mode cpu-steady [--cases subsets | cavity256]: the FP64 oracle's wall time to
residual 1e-8 on the host's cores against the plain FP64 method on the GPU.
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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_bstep_ddc_sweep_256_cavities_f32.traffic.json")
PLUME_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_step_chemotaxis_plume_512x256_f32.traffic.json")
WEIGHTS = os.path.join(ROOT, "paper_2101_03055_amd", "data", "surrogate_ddc128.npz")


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
    return e0.elapsed_time(e1) / 1e3, n_res


# launches before a timed window on a freshly allocated state: the first few
# dozen launches of a 4096^2 step run up to 8 % slower (FP16: 240 us over the
# first 100 launches after 24, 223-225 us from then on)
WARM_LAUNCHES = 200


def kernel_time(step_fn, stream, launches):
    """Mean duration of one step launch: HIP events on the launching stream
    around back-to-back launches (no host synchronisation in between)."""
    import torch

    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    step_fn(launches)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3 / launches


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, phi0, u0, p0, budget_s=15.0, single_s=5.0):
    """The oracle on the host cores: all threads on a ~15 s sample, then one
    thread on a ~5 s sample of the same run (the per-node updates are
    independent, so the thread count does not change results)."""
    from oracle import oracle as O

    o = O.Oracle(wl, phi0, u0, p0)
    o.step(5)  # thread start-up, first touch
    t0 = time.perf_counter()
    o.step(20)
    dt = max(time.perf_counter() - t0, 1e-6) / 20
    steps = max(2, int(budget_s / dt))
    t0 = time.perf_counter()
    o.step(steps)
    el = time.perf_counter() - t0
    lu = wl["nx"] * wl["ny"] * steps
    cores = O.threads()
    O.set_threads(1)
    try:
        o.step(1)
        t0 = time.perf_counter()
        o.step(2)
        dt1 = max(time.perf_counter() - t0, 1e-6) / 2
        s1 = max(2, int(single_s / dt1))
        t0 = time.perf_counter()
        o.step(s1)
        el1 = time.perf_counter() - t0
    finally:
        O.set_threads(cores)
    return {"value": round(lu / el / 1e6, 2), "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "sample": f"{wl['name']}, FP64 oracle, {steps} steps from the same initial state ({el:.1f} s)",
            "single_thread_MLUPS": round(wl["nx"] * wl["ny"] * s1 / el1 / 1e6, 2),
            "single_thread_sample": f"{s1} further steps on one thread ({el1:.1f} s)",
            "cpu_model": cpu_model()}


def traffic_record(path=TRAFFIC_FILE):
    """Counter-measured bytes per launch, if they describe the current kernel sources."""
    try:
        from paper_2101_03055_amd import profsum

        with open(path) as fh:
            rec = json.load(fh)
        if rec.get("source_hash") == profsum.source_hash():
            return rec
    except (OSError, ValueError, KeyError):
        pass
    return None


def hbm_sweep(W, lb, torch):
    out = {}
    for storage in ("f64", "f32", "f16"):
        n = 4096
        wlb, pb, ub, ppb = W.taylor_green_blobs(n=n, steps=0)
        sb = lb.Solver(wlb, pb, ub, ppb, storage=storage, phi_ref=[1.0, 1.0], fp16_scale=1e3, fp16_scale_h=1e4)
        sb.step(WARM_LAUNCHES)
        kt = kernel_time(sb.step, sb.stream, 100)
        bb = bytes_per_lu(2, storage, 0)
        ach = bb * n * n / kt / 1e9
        out[f"{storage}_{n}x{n}"] = {"MLUPS": round(n * n / kt / 1e6, 1), "achieved_GBs": round(ach, 1),
                                     "frac": round(ach / HBM_PEAK_GBS, 4), "mean_launch_us": round(kt * 1e6, 2),
                                     "bytes_per_lu": bb}
        del sb
        torch.cuda.empty_cache()
    # the MRT fluid collision (Lallemand-Luo basis) on the same grid: same bytes, more arithmetic
    for storage in ("f64", "f32"):
        n = 4096
        wlb, pb, ub, ppb = W.taylor_green_blobs(n=n, steps=0)
        wlb = dict(wlb, collision="mrt")
        sb = lb.Solver(wlb, pb, ub, ppb, storage=storage, phi_ref=[1.0, 1.0])
        sb.step(WARM_LAUNCHES)
        kt = kernel_time(sb.step, sb.stream, 100)
        bb = bytes_per_lu(2, storage, 0)
        ach = bb * n * n / kt / 1e9
        out[f"mrt_{storage}_{n}x{n}"] = {"MLUPS": round(n * n / kt / 1e6, 1), "achieved_GBs": round(ach, 1),
                                         "frac": round(ach / HBM_PEAK_GBS, 4), "mean_launch_us": round(kt * 1e6, 2),
                                         "bytes_per_lu": bb}
        del sb
        torch.cuda.empty_cache()
    return out


def cde_sweep(W, lb, torch, n=4096):
    """Case 1 (no fluid): two species in a prescribed cellular flow on n^2,
    periodic, FP64 and FP32.  Algorithmic bytes per lattice update: the 5m
    populations read and written, the prescribed velocity read, the previous
    phi read and written."""
    out = {}
    for storage in ("f64", "f32"):
        wl, phi0, u0, p0 = W.cde_case(n, n, m=2, seed=1)
        s = lb.Solver(wl, phi0, u0, p0, storage=storage, phi_ref=[1.0, 1.0])
        s.step(WARM_LAUNCHES)
        kt = kernel_time(s.step, s.stream, 100)
        b = 8 if storage == "f64" else 4
        bb = 2 * 10 * b + (2 + 2 * 2) * b
        ach = bb * n * n / kt / 1e9
        out[f"{storage}_{n}x{n}"] = {"MLUPS": round(n * n / kt / 1e6, 1), "achieved_GBs": round(ach, 1),
                                     "frac": round(ach / HBM_PEAK_GBS, 4), "mean_launch_us": round(kt * 1e6, 2),
                                     "bytes_per_lu": bb}
        del s
        torch.cuda.empty_cache()
    return out


def sweep_3d(W, torch, n=256):
    """The 3-D path (D3Q7 scalars + D3Q19 fluid, m = 2): periodic Taylor-Green
    vortex carrying two Gaussian blobs on n^3, FP64 and FP32.  Algorithmic
    bytes per lattice update: the 19 + 7m populations read and written."""
    from paper_2101_03055_amd import lb3

    out = {}
    wl, phi0, u0, p0 = W.taylor_green3(n)
    for storage in ("f64", "f32"):
        s = lb3.Solver3(wl, phi0, u0, p0, storage=storage, phi_ref=[1.0, 1.0])
        s.step(WARM_LAUNCHES)
        kt = kernel_time(s.step, s.stream, 40)
        b = 8 if storage == "f64" else 4
        bb = 2 * (19 + 7 * 2) * b
        N = n ** 3
        ach = bb * N / kt / 1e9
        out[f"{storage}_{n}^3"] = {"MLUPS": round(N / kt / 1e6, 1), "achieved_GBs": round(ach, 1),
                                   "frac": round(ach / HBM_PEAK_GBS, 4), "mean_launch_us": round(kt * 1e6, 2),
                                   "bytes_per_lu": bb}
        s.close()
        del s
        torch.cuda.empty_cache()
    return out


def sweep_cases(W):
    """The 256 cavities of the batched sweep (seed 4) and their node count."""
    pds = W.sweep_params(256, seed=4)
    cases = [W.ddc_case(pd) for pd in pds]
    return cases, sum(c[0]["nx"] * c[0]["ny"] for c in cases)


def time_batch(b, steps, window=1000):
    """Wall time of exactly `steps` batched steps on the batch's stream; every
    full window of `window` steps runs through lbb_run (the steady sweep's
    loop: snapshot, steps, FP64 per-cavity residual), a shorter remainder as
    plain steps.  Returns (seconds, residual evaluations)."""
    import torch

    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    done = n_res = 0
    e0.record(b.stream)
    while done < steps:
        k = min(window, steps - done)
        if k == window:
            b.run(tol=1e-300, check_every=window, max_steps=window)  # never converges: all cavities keep running
            n_res += 1
        else:
            b.step(k)
        done += k
    e1.record(b.stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3, n_res


def tiles_by_width(b, cases):
    """The autotuned tile shape of each cavity width ({nx: [tile_x, tile_y]})."""
    out = {}
    for i, c in enumerate(cases):
        out[str(c[0]["nx"])] = list(b.cavity_tile(i))
    return dict(sorted(out.items(), key=lambda kv: int(kv[0])))


def batch_headline(W, lb, torch, steps, warmup):
    """The batched sweep: autotune, warm up, time `steps` steps, then the
    step kernel's mean launch duration and a 2000-step production run."""
    cases, nodes = sweep_cases(W)
    b = lb.Batch(cases, storage="f32", phi_ref=[0.5, 0.5])
    tx, ty, us = b.autotune(10)
    by_width = tiles_by_width(b, cases)
    b.step(warmup + (warmup & 1))
    el, n_res = time_batch(b, steps)
    kt = kernel_time(b.step, b.stream, 256)
    el_prod, n_prod = time_batch(b, 2000)
    st = [b.time(i)[1] for i in range(b.count)]
    return b, {"cases": cases, "nodes": nodes, "tile": [tx, ty], "tiles_by_width": by_width, "autotune_us": round(us, 2),
               "elapsed": el, "residual_evals": n_res, "kernel_s": kt,
               "production_run": {"steps": 2000, "residual_windows": n_prod, "seconds": round(el_prod, 4),
                                  "MLUPS": round(nodes * 2000 / el_prod / 1e6, 1),
                                  "note": "lbb_run windows of 1000 steps: snapshot + steps + FP64 residual of "
                                          "every cavity"},
               "diverged": sum(1 for v in st if v == 2)}


def cpu_baseline_sweep(W, cases, stride=16, budget_s=15.0):
    """The FP64 oracle on every `stride`-th cavity of the sweep (all host
    threads), the same number of steps on each, sized to ~budget_s seconds."""
    from oracle import oracle as O

    sub = cases[::stride]
    nodes = sum(c[0]["nx"] * c[0]["ny"] for c in sub)
    probe = O.Oracle(*sub[0])
    probe.step(3)
    t0 = time.perf_counter()
    probe.step(10)
    rate = sub[0][0]["nx"] * sub[0][0]["ny"] * 10 / max(time.perf_counter() - t0, 1e-6)
    del probe
    steps = max(2, int(budget_s * rate / nodes))
    el = 0.0
    for c in sub:
        o = O.Oracle(*c)
        t0 = time.perf_counter()
        o.step(steps)
        el += time.perf_counter() - t0
        del o
    sizes = sorted({c[0]["nx"] for c in sub})
    return {"value": round(nodes * steps / el / 1e6, 2), "unit": "MLUPS", "cores": O.threads(), "kind": "oracle",
            "sample": f"ddc_sweep_256_cavities: cavities 0, {stride}, ..., {stride * (len(sub) - 1)} "
                      f"({len(sub)} of 256, sides {sizes[0]}..{sizes[-1]}, {nodes} nodes), {steps} steps each "
                      f"from rest, FP64 oracle ({el:.1f} s)",
            "cpu_model": cpu_model()}


def oracle_to_steady(case, tol=1e-8, check_every=1000, max_steps=3_000_000, log=None):
    """The FP64 CPU oracle from the case's initial state to the steady
    criterion lb_solve_steady uses (every check_every steps: sum |q - q_prev| /
    sum |q| below tol for u_x, u_y and every phi).  Returns (steps, seconds)."""
    from oracle import oracle as O

    o = O.Oracle(*case)
    prev = None
    t0 = time.perf_counter()
    while o.t < max_steps:
        o.step(check_every)
        phi, u, _ = o.moments()
        cur = [u[0], u[1], *phi]
        if prev is not None:
            res = max(float(np.abs(a - b).sum() / max(np.abs(a).sum(), 1e-300)) for a, b in zip(cur, prev))
            if log and o.t % (100 * check_every) == 0:
                log(f"  oracle {o.t} steps, {time.perf_counter() - t0:.0f} s, residual {res:.2e}")
            if res < tol:
                break
        prev = cur
    return o.t, time.perf_counter() - t0


def cpu_steady(W, lb, torch, which):
    """Wall time to residual 1e-8, the FP64 oracle on the host's cores against
    the plain FP64 method on the GPU (one cavity at a time, step graphs), on
    the same seeded cases: 'cavity256' = the 256^2 double-diffusive cavity
    (Ra 1e5, Pr 0.71, Le 2, N 1, Sr = Df = 0.1) in full; 'subsets' = the two
    64^2 cavities of the 256-cavity sweep and two 128^2 held-out cavities of the
    surrogate study (seeds 20001, 20006) from rest (the sweep's pair: of its
    first eight 64^2 cavities, the two the GPU brings to 1e-8 fastest; needs
    the GPU)."""
    from oracle import oracle as O

    log = lambda m: print(m, file=sys.stderr, flush=True)
    if which == "cavity256":
        named = [("ddc_cavity_256", W.ddc_cavity(256))]
    else:
        cases, _ = sweep_cases(W)
        # of the first eight 64^2 cavities, the two that the GPU brings to 1e-8 in the fewest
        # steps (some of the sweep's cavities are unsteady or take millions of steps)
        found = []
        for i in [i for i, c in enumerate(cases) if c[0]["nx"] == 64][:8]:
            g = lb.Solver(*cases[i], storage="f64")
            steps, _, st = g.solve_steady(1e-8, 1000, 600_000)
            g.close()
            if st == lb.LB_OK:
                found.append((steps, i))
        small = [i for _, i in sorted(found)[:2]]
        named = [(f"ddc_sweep_256_cavities[{i}] ({cases[i][0]['nx']}x{cases[i][0]['ny']})", cases[i]) for i in small]
        named += [(f"surrogate held-out seed {s} (128x128)", W.ddc_case(W.sweep_case(s, 128))) for s in (20001, 20006)]
    out = []
    for name, case in named:
        nodes = case[0]["nx"] * case[0]["ny"]
        rec = {"case": name, "nodes": nodes}
        if lb is not None:
            log(f"{name}: GPU plain FP64")
            g = lb.Solver(*case, storage="f64")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            gsteps, _, gst = g.solve_steady(1e-8, 1000, 3_000_000)
            torch.cuda.synchronize()
            gsec = time.perf_counter() - t0
            g.close()
            rec.update({"gpu_steps": gsteps, "gpu_converged": gst == lb.LB_OK, "gpu_seconds": round(gsec, 3)})
            log(f"{name}: GPU {gsteps} steps {gsec:.2f} s")
        log(f"{name}: oracle ({O.threads()} threads)")
        osteps, osec = oracle_to_steady(case, log=log)
        rec.update({"oracle_steps": osteps, "oracle_seconds": round(osec, 1),
                    "oracle_MLUPS": round(nodes * osteps / osec / 1e6, 2)})
        if "gpu_seconds" in rec:
            rec["speedup"] = round(osec / rec["gpu_seconds"], 1)
        out.append(rec)
        log(json.dumps(out[-1]))
    return {"cases": out, "oracle_threads": O.threads(), "cpu_model": cpu_model(),
            "criterion": "residual 1e-8 (sum |q - q_prev| / sum |q| over 1000 steps, u_x, u_y, phi)"}


def steady_warm_vs_cold(W, torch, n_cases=16, max_steps=600_000, n_plain=4):
    """Warm vs cold steady solves (batched FP32 phase + FP64 finish to 1e-8),
    and the plain FP64 method on the first n_plain cavities both converged."""
    from paper_2101_03055_amd import sg, surrogate_study as SS

    if not os.path.exists(WEIGHTS):
        return None
    net = sg.Surrogate(16, 128, 128)
    net.set_weights(np.load(WEIGHTS)["w"])
    seeds = list(range(20000, 20000 + n_cases))
    pds = [W.sweep_case(s, 128) for s in seeds]
    cases = [W.ddc_case(pd) for pd in pds]
    params = np.array([W.normalise(pd) for pd in pds], dtype=np.float32)
    quiet = lambda s: None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pred = SS.predict(net, params)
    t_pred = time.perf_counter() - t0
    warm, fw = SS.solve_path(cases, pred, max_steps=max_steps, label="warm", log=quiet)
    cold, fc = SS.solve_path(cases, None, max_steps=max_steps, label="cold", log=quiet)
    ok = [i for i in range(n_cases) if warm["status"][i] == 1 and cold["status"][i] == 1]
    # the plain method (FP64, one cavity at a time, from rest) on the first few converged cavities
    plain_s, plain_err = [], []
    for i in ok[:n_plain]:
        _, _, secs, f = SS.plain_solve(cases[i])
        plain_s.append(secs)
        plain_err.append(SS.rel_l2(fw[i], f))
    per_warm = (warm["seconds"] + t_pred) / n_cases
    # time to steady: a batch's wall time is set by its slowest cavity, and
    # cavities that never become steady (oscillating flows, e.g. Nc near -1)
    # run to the step cap either way.  Time the warm and the cold path again
    # on the cavities that became steady in either run above, with a higher
    # cap, so that both times measure the approach to a steady state.
    steady = [i for i in range(n_cases) if warm["status"][i] == 1 or cold["status"][i] == 1]
    sub = [cases[i] for i in steady]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pred_s = SS.predict(net, params[steady])
    t_pred_s = time.perf_counter() - t0
    warm_s, _ = SS.solve_path(sub, pred_s, max_steps=2 * max_steps, label="warm", log=quiet)
    cold_s, _ = SS.solve_path(sub, None, max_steps=2 * max_steps, label="cold", log=quiet)
    to_steady = {"cavities": len(steady), "max_steps_per_phase": 2 * max_steps,
                 "steady_warm": sum(1 for v in warm_s["status"] if v == 1),
                 "steady_cold": sum(1 for v in cold_s["status"] if v == 1),
                 "wall_s_warm": round(warm_s["seconds"] + t_pred_s, 2), "wall_s_cold": round(cold_s["seconds"], 2),
                 "speedup": round(cold_s["seconds"] / (warm_s["seconds"] + t_pred_s), 3)}
    if plain_s:
        per = (warm_s["seconds"] + t_pred_s) / len(steady)
        to_steady["warm_s_per_cavity"] = round(per, 3)
        to_steady["speedup_vs_plain"] = round(float(np.mean(plain_s)) / per, 2)
    return {"cases": n_cases, "L": 128, "converged_both": len(ok), "tol": 1e-8,
            "time_to_steady": to_steady,
            "plain_fp64_s_per_case": round(float(np.mean(plain_s)), 3) if plain_s else None,
            "warm_batched_s_per_case": round(per_warm, 3),
            "speedup_vs_plain": round(float(np.mean(plain_s)) / per_warm, 2) if plain_s else None,
            "warm_relL2_vs_plain_max": max(plain_err, default=None),
            "wall_s_warm": round(warm["seconds"] + t_pred, 2), "wall_s_cold": round(cold["seconds"], 2),
            "speedup": round(cold["seconds"] / (warm["seconds"] + t_pred), 3),
            "steps_warm_median": float(np.median([warm["steps_total"][i] for i in ok])) if ok else None,
            "steps_cold_median": float(np.median([cold["steps_total"][i] for i in ok])) if ok else None,
            "warm_relL2_vs_cold_max": max((SS.rel_l2(fw[i], fc[i]) for i in ok), default=None),
            "note": "cavities that do not become steady within the cap (e.g. Nc near -1) count in both batched "
                    "wall times; per-case batched time = batch wall time / cases"}


def surrogate_bench(torch, epochs=4, samples=64):
    """Training and inference throughput of the CNN surrogate (BF16 MFMA
    convolutions) at batch 16 on 128 x 128, random weights and targets.
    Algorithmic flops per training step: forward, data gradient (all layers
    but the first) and weight gradient of every 3x3 convolution over the real
    (unpadded) channels, 2 flops per multiply-add."""
    from paper_2101_03055_amd import sg

    B, H, Wd = 16, 128, 128
    macs = [9 * sg.layer_info(l)[0] * sg.layer_info(l)[1] for l in range(sg.SG_LAYERS)]
    flops_step = 2.0 * B * H * Wd * (2 * sum(macs) + sum(macs[1:]))
    net = sg.Surrogate(B, H, Wd)
    net.set_weights(sg.init_weights(0))
    g = torch.Generator(device="cpu").manual_seed(0)
    dp = torch.rand((samples, 5), generator=g).cuda()
    df = (0.1 * torch.randn((samples, 4, H, Wd), generator=g)).cuda()
    net.train_epochs(dp, df, samples, 1)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    steps = epochs * samples // B
    reps = []
    for _ in range(5):  # the median of five timed runs of `epochs` epochs
        e0.record(net.stream)
        net.train_epochs(dp, df, samples, epochs)
        e1.record(net.stream)
        torch.cuda.synchronize()
        reps.append(e0.elapsed_time(e1) / 1e3 / steps)
    t_step = float(np.median(reps))
    out = torch.empty((B, 4, H, Wd), device="cuda")
    net.predict(dp, B, out)
    torch.cuda.synchronize()
    e0.record(net.stream)
    for _ in range(10):
        net.predict(dp, B, out)
    e1.record(net.stream)
    torch.cuda.synchronize()
    t_pred = e0.elapsed_time(e1) / 1e3 / 10
    flops_pred = 2.0 * B * H * Wd * sum(macs)
    layers = surrogate_kernel_rooflines(net, torch, B, H, Wd)
    bound_step = sum(k["binding_us"] for L in layers for k in L["kernels"].values()) * 1e-6
    return {"batch": B, "grid": [H, Wd], "train_step_ms": round(t_step * 1e3, 3),
            "train_TFLOPs": round(flops_step / t_step / 1e12, 1),
            "train_frac_bf16_peak": round(flops_step / t_step / 2.5e15, 4),
            "train_binding_roofline_ms": round(bound_step * 1e3, 3),
            "train_frac_binding_roofline": round(bound_step / t_step, 4),
            "predict_ms_per_batch": round(t_pred * 1e3, 3),
            "predict_TFLOPs": round(flops_pred / t_pred / 1e12, 1),
            "kernels": layers,
            "note": "binding roofline per kernel = max(algorithmic HBM bytes / 8 TB/s, real-channel flops / "
                    "2.5 PFLOP/s); bytes are the stored (padded) tensors read and written once: forward x in, "
                    "z (FP32) and y out; data gradient dz and z_prev in, dx out; weight gradient dz and x in, "
                    "dW out (the split-K partial sums are not counted)"}


def surrogate_kernel_rooflines(net, torch, B, H, Wd, reps=10):
    """Each convolution of the training pass timed alone through sg_conv /
    sg_weight_grad (HIP events on the surrogate's stream, `reps` back-to-back
    calls) against its binding roofline."""
    from paper_2101_03055_amd import sg

    P = B * H * Wd
    g = torch.Generator(device="cpu").manual_seed(5)
    out = []
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0.record(net.stream)
        for _ in range(reps):
            fn()
        e1.record(net.stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e3 / reps  # us

    for l in range(sg.SG_LAYERS):
        cin, cout, ci, co = sg.layer_info(l)
        x = (torch.rand((B, H, Wd, ci), generator=g) - 0.5).to(torch.bfloat16).cuda()
        gz = (torch.rand((B, H, Wd, co), generator=g) - 0.5).to(torch.bfloat16).cuda()
        z = torch.empty((B, H, Wd, co), dtype=torch.float32, device="cuda")
        y = torch.empty((B, H, Wd, co), dtype=torch.bfloat16, device="cuda")
        zp = torch.rand((B, H, Wd, ci), generator=g).cuda()
        dx = torch.empty((B, H, Wd, ci), dtype=torch.bfloat16, device="cuda")
        dw = torch.empty((co, 9, ci), dtype=torch.float32, device="cuda")
        db = torch.empty((co,), dtype=torch.float32, device="cuda")
        gemm = 2.0 * P * 9 * cin * cout
        kern = {}
        kern["forward"] = (timed(lambda: net.conv(l, 0, B, x, y, d_z=z)), gemm, P * (2 * ci + 6 * co))
        if l > 0:
            kern["data_gradient"] = (timed(lambda: net.conv(l, 1, B, gz, dx, d_zprev=zp)), gemm, P * (2 * co + 6 * ci))
        kern["weight_gradient"] = (timed(lambda: net.weight_grad(l, B, gz, x, dw, db)), gemm,
                                   P * (2 * co + 2 * ci) + 4 * 9 * co * ci)
        rec = {"layer": l, "channels": [cin, cout], "kernels": {}}
        for k, (us, fl, by) in kern.items():
            bind = max(by / 8e12, fl / 2.5e15) * 1e6
            rec["kernels"][k] = {"us": round(us, 2), "TFLOPs": round(fl / us / 1e6, 1),
                                 "GBs": round(by / us / 1e3, 1), "binding_us": round(bind, 2),
                                 "bound": "hbm" if by / 8e12 >= fl / 2.5e15 else "mfma",
                                 "frac_binding": round(bind / us, 4)}
        out.append(rec)
        del x, gz, z, y, zp, dx
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--cases", choices=["subsets", "cavity256"], default="subsets",
                    help="cpu-steady: which cases the oracle solves to residual 1e-8")
    ap.add_argument("--mode", choices=["bench", "pmc", "copy", "sweep", "batch", "plume", "surrogate", "cde", "3d",
                                       "cpu-steady"],
                    default="bench",
                    help="pmc: only the plume's step kernel (for counter runs); "
                         "copy: a plain 1 GiB device copy to calibrate the byte counters; "
                         "batch / plume / sweep / surrogate / cde / 3d: one leg only (for profiles)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(the design notes describe how the domain would be sharded).", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2101_03055_amd import lb, workloads as W

    if args.mode == "cpu-steady" and not torch.cuda.is_available():
        # a host without a GPU: the oracle's side alone
        print(json.dumps({"cpu_steady": cpu_steady(W, None, None, args.cases)}), flush=True)
        return
    torch.cuda.set_device(0)
    if args.mode == "copy":
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")  # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": src.numel() * 4, "copies": 5}), flush=True)
        return
    if args.mode == "sweep":
        print(json.dumps({"hbm_sweep": hbm_sweep(W, lb, torch)}), flush=True)
        return
    if args.mode == "cde":
        print(json.dumps({"cde_sweep": cde_sweep(W, lb, torch)}), flush=True)
        return
    if args.mode == "cpu-steady":
        print(json.dumps({"cpu_steady": cpu_steady(W, lb, torch, args.cases)}), flush=True)
        return
    if args.mode == "surrogate":
        print(json.dumps({"surrogate": surrogate_bench(torch)}), flush=True)
        return
    if args.mode == "3d":
        print(json.dumps({"sweep_3d": sweep_3d(W, torch)}), flush=True)
        return
    if args.mode == "batch":
        cases, nodes = sweep_cases(W)
        b = lb.Batch(cases, storage="f32", phi_ref=[0.5, 0.5])
        tx, ty, _ = b.autotune(10)  # 7 shapes for all cavities, then per width, each 2 + 10 steps
        tuned = b.time(0)[0]
        kt = kernel_time(b.step, b.stream, 256)
        print(json.dumps({"launches": tuned + 256, "timed_launches": 256, "tile": [tx, ty],
                          "tiles_by_width": tiles_by_width(b, cases),
                          "mean_launch_us": round(kt * 1e6, 2),
                          "bytes_per_launch": bytes_per_lu(2, "f32", 0) * nodes}), flush=True)
        return
    if args.mode == "plume":
        print(json.dumps({"plume": plume(W, lb, torch, 4000, 200)}), flush=True)
        return
    if args.mode == "pmc":
        wl, phi0, u0, p0 = W.chemotaxis_plume()
        solver = lb.Solver(wl, phi0, u0, p0, storage="f32", phi_ref=[1.0, 1.0])
        solver.step(200)
        torch.cuda.synchronize()
        print(json.dumps({"pmc_steps": 200, "bytes_per_launch": bytes_per_lu(2, "f32", 1) * wl["nx"] * wl["ny"]}),
              flush=True)
        return

    b, r = batch_headline(W, lb, torch, args.steps, args.warmup)
    nodes = r["nodes"]
    bpl = bytes_per_lu(2, "f32", 0)
    kt = r["kernel_s"]
    achieved = bpl * nodes / kt / 1e9
    tr = traffic_record()
    el = r["elapsed"]
    out = {
        "metric": METRIC, "value": round(nodes * args.steps / el / 1e6, 1), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded sweep law; cavities start from rest as in Sec. 3.2)",
        "config": {"workload": "ddc_sweep_256_cavities", "cavities": 256, "sides": "64..256 step 32",
                   "nodes": nodes, "state_MB": round(nodes * 19 * 4 / 1e6, 1), "m": 2,
                   "storage": "f32 deviations from phi_ref = (0.5, 0.5) and rho0", "collision": "bgk",
                   "tile": r["tile"], "tiles_by_width": r["tiles_by_width"], "residual_every": 1000,
                   "residual_evals_timed": r["residual_evals"]},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": round(tr["traffic_bytes_per_launch"]) if tr else None,
                     "kernel": "k_bstep (even/odd AA-pattern launches alternate)",
                     "bytes_per_launch": bpl * nodes, "bytes_per_node": bpl, "mean_launch_us": round(kt * 1e6, 3)},
        "production_run": r["production_run"],
        "diverged_cavities": r["diverged"],
    }
    cases = r["cases"]
    b.close()
    del b
    torch.cuda.empty_cache()
    if not args.no_extra:
        out["plume"] = plume(W, lb, torch, 4000, 200)
        out["hbm_sweep"] = hbm_sweep(W, lb, torch)
        out["cde_sweep"] = cde_sweep(W, lb, torch)
        torch.cuda.empty_cache()
        out["sweep_3d"] = sweep_3d(W, torch)
        out["steady_warm_vs_cold"] = steady_warm_vs_cold(W, torch)
        out["surrogate"] = surrogate_bench(torch)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline_sweep(W, cases)
    print(json.dumps(out), flush=True)


def plume(W, lb, torch, steps, warmup):
    """The chemotaxis-fluid plume 512 x 256 (FP32 and FP64): its 21 MB state
    stays in the MALL, so its rates are cache-resident, not HBM-bound."""
    wl, phi0, u0, p0 = W.chemotaxis_plume()
    N = wl["nx"] * wl["ny"]
    bpl = bytes_per_lu(2, "f32", 1)
    solver = lb.Solver(wl, phi0, u0, p0, storage="f32", phi_ref=[1.0, 1.0])
    el, n_res = time_steps(solver, steps, warmup)
    kt = kernel_time(solver.step, solver.stream, 1024)
    tr = traffic_record(PLUME_TRAFFIC_FILE)
    out = {"workload": wl["name"], "nx": wl["nx"], "ny": wl["ny"], "steps": steps, "residual_evals": n_res,
           "MLUPS": round(N * steps / el / 1e6, 1), "mean_launch_us": round(kt * 1e6, 3),
           "bytes_per_launch": bpl * N, "effective_GBs": round(bpl * N / kt / 1e9, 1),
           "traffic": round(tr["traffic_bytes_per_launch"]) if tr else None,
           "bound": "cache-resident (21 MB state in the 256 MB MALL)"}
    s64 = lb.Solver(wl, phi0, u0, p0, storage="f64")
    el64, _ = time_steps(s64, 2000, 100)
    kt64 = kernel_time(s64.step, s64.stream, 512)
    out["fp64"] = {"MLUPS": round(N * 2000 / el64 / 1e6, 1), "mean_launch_us": round(kt64 * 1e6, 3),
                   "effective_GBs": round(bytes_per_lu(2, "f64", 1) * N / kt64 / 1e9, 1)}
    return out


if __name__ == "__main__":
    main()
