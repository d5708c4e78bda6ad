"""Influence of the chemotaxis parameters (Sec. 3.1.2): vertical profiles of
the bacteria and oxygen concentrations at t = 0.22 for the sweeps the paper
describes, all run together as one batch on the GPU (FP64).

Cases (gamma = 418, Sc = 7700, dt = 1e-8, regularised r(c) with eps = dx,
c* = 0.3, initial layer n0 = 1 above y = 0.501 - 0.01 sin((x - 0.5) pi) and
0.5 below, c0 = 1, u0 = 0):
  base   alpha = 5, beta = 5, delta = 0.25 (the comparison case of the section);
  alpha  1, 2, 4, 5.952 with beta = 10, delta = 1;
  beta   7.2296, 10, 20, 40 with alpha = 5, delta = 1;
  delta  1, 5, 10, 15 (the values of the text) and 25 (the caption's last
         value) with alpha = beta = 10.
The grid is the paper's dx = 0.02 (50 rows) on one period of the modulation,
x in [-1, 1], periodic in x (the section does not repeat the domain; with
data and lattice symmetric about x = 0 and of period 2 in x, a wider periodic
box would hold copies of the same solution).

The paper's figures are not in the text, so the runs are checked against
what the text states (trends with alpha, beta and delta) and against what the
equations fix: the bacteria total is conserved (no-flux walls, no bacteria
source) and the solution stays mirror symmetric about x = 0.

``python -m paper_2101_03055_amd.param_study --out FILE`` writes the profiles
and trend measures as JSON.
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import lb, workloads as W

T_END = 0.22

CASES = [("base", 5.0, 5.0, 0.25)]
CASES += [(f"alpha={a:g}", a, 10.0, 1.0) for a in (1.0, 2.0, 4.0, 5.952)]
CASES += [(f"beta={b:g}", 5.0, b, 1.0) for b in (7.2296, 10.0, 20.0, 40.0)]
CASES += [(f"delta={d:g}", 10.0, 10.0, d) for d in (1.0, 5.0, 10.0, 15.0, 25.0)]


def measures(phi, u, y):
    """x-averaged profiles and the scalar measures the trends are stated in."""
    n, c = phi[0], phi[1]
    npro, cpro = n.mean(axis=1), c.mean(axis=1)
    top = y > 0.9
    low = y < 0.5
    return {
        "n_profile": npro.tolist(), "c_profile": cpro.tolist(),
        "n_top": float(npro[top].mean()),          # bacteria under the surface (top tenth)
        "n_surface": float(npro[y > 0.95].mean()), # bacteria gathered at the surface (top 5 %)
        "n_lower_half": float(npro[low].mean()),   # bacteria left in the lower half
        "c_mean": float(c.mean()),                 # oxygen left in the domain
        "c_lower_half": float(cpro[low].mean()),
        "c_min": float(c.min()),
        "u_max": float(np.sqrt(u[0] ** 2 + u[1] ** 2).max()),
        "mirror_asymmetry": float(max(np.abs(n - n[:, ::-1]).max(), np.abs(c - c[:, ::-1]).max())),
    }


def run(nx=100, ny=50, dt=1e-8, t_end=T_END, cases=CASES, log=print):
    built = [W.chemotaxis_layer(a, b, d, nx=nx, ny=ny, a=nx / (2.0 * ny), dt=dt) for _, a, b, d in cases]
    batch = lb.Batch(built, storage="f64")
    steps = int(round(t_end / dt))
    n_total0 = [float(c[1][0].sum()) for c in built]
    t0 = time.perf_counter()
    done, chunk = 0, 1_000_000
    while done < steps:
        k = min(chunk, steps - done)
        batch.step(k)
        done += k
        _, _, _ = batch.moments(0)   # synchronises; progress point
        log(f"  {done} / {steps} steps ({time.perf_counter() - t0:.1f} s)")
    seconds = time.perf_counter() - t0
    y = (np.arange(ny) + 0.5) / ny
    out = {"t": t_end, "dt": dt, "steps": steps, "nx": nx, "ny": ny, "dx": 1.0 / ny, "x_range": [-nx / (2.0 * ny),
           nx / (2.0 * ny)], "seconds": round(seconds, 2), "gamma": 418.0, "Sc": 7700.0, "cstar": 0.3,
           "y": y.tolist(), "cases": []}
    for i, (label, a, b, d) in enumerate(cases):
        phi, u, _ = batch.moments(i)
        rec = {"label": label, "alpha": a, "beta": b, "delta": d,
               "tau_n": 0.5 + 3 * built[i][0]["D"][0][0], "tau_c": 0.5 + 3 * built[i][0]["D"][1][1],
               "tau_f": built[i][0]["tau_f"],
               "n_total_rel_change": float(phi[0].sum() / n_total0[i] - 1.0)}
        rec.update(measures(phi, u, y))
        out["cases"].append(rec)
    batch.close()
    return out


def sweep(out, name):
    """The cases of one sweep in parameter order."""
    return [c for c in out["cases"] if c["label"].startswith(name + "=")]


def statements(out):
    """The measures behind each statement of the section, per sweep in
    parameter order (alpha: 1, 2, 4, 5.952; beta: 7.2296, 10, 20, 40; delta:
    1, 5, 10, 15, 25), and the base case's profiles."""
    y = np.asarray(out["y"])
    get = lambda name, key: [c[key] for c in sweep(out, name)]
    base = next(c for c in out["cases"] if c["label"] == "base")
    nb, cb = np.asarray(base["n_profile"]), np.asarray(base["c_profile"])
    return {
        # alpha: more bacteria near the surface, fewer left below, less oxygen consumed below
        "alpha_n_top": get("alpha", "n_top"), "alpha_n_lower_half": get("alpha", "n_lower_half"),
        "alpha_c_lower_half": get("alpha", "c_lower_half"),
        # beta: less oxygen at every height, more bacteria swimming up to the surface
        "beta_c_profiles": [c["c_profile"] for c in sweep(out, "beta")], "beta_n_surface": get("beta", "n_surface"),
        # delta: oxygen fills the domain, bacteria stay below, fewer swim up
        "delta_c_mean": get("delta", "c_mean"), "delta_n_lower_half": get("delta", "n_lower_half"),
        "delta_n_top": get("delta", "n_top"),
        # base: below the cut-off level the bacteria increase towards the bottom
        "base_n_lower": nb[y < 0.5].tolist(), "base_c_bottom": float(cb[0]),
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    out = run()
    for c in out["cases"]:
        print(json.dumps({k: c[k] for k in ("label", "n_top", "n_lower_half", "c_mean", "c_lower_half", "c_min",
                                            "u_max", "n_total_rel_change", "mirror_asymmetry")}), flush=True)
    if args.out:
        with open(args.out, "w") as fh:
            json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
