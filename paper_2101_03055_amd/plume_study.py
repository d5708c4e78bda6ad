"""Plumes from a sinusoidally modulated bacteria layer (Sec. 3.1.3, beta = 10,
gamma = 1000): the chemotaxis-fluid system run on the GPU to t = 1 with
snapshots at the times the paper describes.

The paper's figures are not available, so the run is checked against the
statements of its text that can be measured:
 * the instability starts at the lower edge of the dense layer (t = 0.2);
 * plumes have formed by t = 0.3 and reach the bottom around t = 0.4;
 * at t = 0.5 the oxygen stays above the cut-off c* = 0.3 everywhere;
plus what the equations fix: the bacteria total is conserved (no-flux walls,
no source), and the initial data are mirror symmetric about x = 0, which the
scheme preserves up to rounding (the lattice is symmetric under x -> -x).

``python -m paper_2101_03055_amd.plume_study --out DIR`` runs the cases of
CASES and writes summary.json (and the snapshots, fields_<case>.npz) to DIR.
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np

from . import lb, workloads as W

TIMES = (0.1, 0.2, 0.3, 0.4, 0.5, 0.75, 1.0)


def count_plumes(n, y, frac=0.25):
    """Plumes = separate x-intervals where the bacteria density averaged over
    the lower half (y < 0.45) exceeds the mean by frac of its x-range; the
    x-axis is periodic."""
    prof = n[y < 0.45].mean(axis=0)
    lo, hi = prof.min(), prof.max()
    if hi - lo < 1e-6:
        return 0, prof
    above = prof > prof.mean() + frac * (hi - lo)
    if above.all():
        return 1, prof
    # count rising edges on the periodic axis
    return int(np.sum(above & ~np.roll(above, 1))), prof


def snapshot(phi, u, y, dx, n_total0):
    n, c = phi[0], phi[1]
    nplumes, prof = count_plumes(n, y)
    # lowest row where the layer has spread: first row from the bottom whose
    # x-max exceeds the initial lower density 0.5 by 10 %
    rows = np.where(n.max(axis=1) > 0.55)[0]
    front = float(y[rows.min()]) if rows.size else 1.0
    return {
        "n_total_rel_change": float(n.sum() / n_total0 - 1.0),
        "c_min": float(c.min()),
        "n_min": float(n.min()),
        "n_max": float(n.max()),
        "u_max": float(np.sqrt(u[0] ** 2 + u[1] ** 2).max()),
        "plumes": nplumes,
        "front_height": front,
        "n_bottom_max": float(n[y < 0.05].max()),
        "mirror_asymmetry": float(np.abs(n - n[:, ::-1]).max()),
        "x_std_lower_half": float(prof.std()),
    }


# (label, nx, ny, dt, a): the paper's grid and step on [-3, 3] (Secs. 3.1.1,
# 3.1.3), the same at half the spacing (same dt/dx^2), and a [-1, 1] box
CASES = (("paper_6x1_dx0.02", 300, 50, 2.5e-7, 3.0),
         ("refined_6x1_dx0.01", 600, 100, 6.25e-8, 3.0),
         ("narrow_2x1_dx0.0078", 256, 128, 1e-7, 1.0))


def run(nx=300, ny=50, dt=2.5e-7, a=3.0, storage="f64", times=TIMES, out=None, label=None):
    wl, phi0, u0, p0 = W.chemotaxis_sinusoidal(nx, ny, dt, a)
    dx = 1.0 / ny
    y = (np.arange(ny) + 0.5) * dx
    s = lb.Solver(wl, phi0, u0, p0, storage=storage, phi_ref=None if storage == "f64" else [0.75, 1.0])
    n_total0 = float(phi0[0].sum())
    snaps, fields = [], {}
    t0 = time.perf_counter()
    done = 0
    for t in times:
        target = int(round(t / dt))
        s.step(target - done)
        done = target
        phi, u, _ = s.moments()
        rec = {"t": t, "steps": done, "seconds": time.perf_counter() - t0}
        rec.update(snapshot(phi, u, y, dx, n_total0))
        snaps.append(rec)
        fields[f"n_t{t}"] = phi[0].astype(np.float32)
        fields[f"c_t{t}"] = phi[1].astype(np.float32)
        print(json.dumps(rec), flush=True)
    summary = {
        "case": label or wl["name"], "nx": nx, "ny": ny, "domain_x": [-a, a], "dx": dx, "dt": dt, "storage": storage,
        "tau_f": wl["tau_f"], "tau_n": 0.5 + 3 * wl["D"][0][0], "tau_c": 0.5 + 3 * wl["D"][1][1],
        "parameters": {"alpha": 10.0, "beta": 10.0, "delta": 5.0, "gamma": 1000.0, "Sc": 500.0, "cstar": 0.3},
        "snapshots": snaps,
    }
    if out:
        os.makedirs(out, exist_ok=True)
        np.savez_compressed(os.path.join(out, f"fields_{summary['case']}.npz"), **fields)
    return summary


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--out", default=None)
    ap.add_argument("--storage", default="f64")
    args = ap.parse_args()
    results = []
    for label, nx, ny, dt, a in CASES:
        print(f"== {label}: {nx} x {ny}, dt {dt}, x in [-{a}, {a}]", flush=True)
        results.append(run(nx, ny, dt, a, args.storage, out=args.out, label=label))
    if args.out:
        with open(os.path.join(args.out, "summary.json"), "w") as fh:
            json.dump({"cases": results}, fh, indent=1)


if __name__ == "__main__":
    main()
