"""What the trained surrogate gains: steady double-diffusive cavities (128^2,
held-out parameter draws of the sweep law) solved by the plain FP64 method
from rest and from the network's prediction, both to residual 1e-8.

The weights were trained by surrogate_study.py on 1604 LB steady states of
the same law (seeds 10000..11999; these tests use seeds from 20000 on).
"""
import os

import numpy as np
import pytest

from paper_2101_03055_amd import lb, sg, surrogate_study as SS, workloads as W

pytestmark = pytest.mark.gpu

WEIGHTS = os.path.join(os.path.dirname(SS.__file__), "data", "surrogate_ddc128.npz")
CASES = [1, 3, 5, 9]


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def fields(s):
    phi, u, _ = s.moments()
    return np.stack([u[0] / SS.U_LAT, u[1] / SS.U_LAT, phi[0], phi[1]])


@pytest.fixture(scope="module")
def predictions():
    net = sg.Surrogate(len(CASES), 128, 128)
    net.set_weights(np.load(WEIGHTS)["w"])
    pds = [W.sweep_case(20000 + k, 128) for k in CASES]
    params = np.array([W.normalise(pd) for pd in pds], dtype=np.float32)
    return pds, SS.predict(net, params)


def test_warm_start_saves_steps_and_reaches_the_plain_solution(predictions):
    pds, pred = predictions
    total_cold = total_warm = 0
    for pd, pf in zip(pds, pred):
        case = W.ddc_case(pd)
        cold = lb.Solver(*case)
        n_cold, _, st_cold = cold.solve_steady(1e-8, 1000, 3_000_000)
        fc = fields(cold)
        wl = case[0]
        warm = lb.Solver(wl, np.stack([pf[2], pf[3]]), np.stack([pf[0], pf[1]]) * SS.U_LAT, None)
        n_warm, _, st_warm = warm.solve_steady(1e-8, 1000, 3_000_000)
        fw = fields(warm)
        e_pred, e_warm = rel(pf, fc), rel(fw, fc)
        print(f"Ra {pd['Ra']:.3g} Le {pd['Le']:.2f} Nc {pd['Nc']:.2f}: cold {n_cold} steps, warm {n_warm} steps, "
              f"prediction relL2 {e_pred:.2e}, warm result relL2 {e_warm:.2e}", flush=True)
        assert st_cold == lb.LB_OK and st_warm == lb.LB_OK
        assert e_pred < 0.03          # the network learned the steady fields
        assert e_warm < 1e-5          # the LB iteration judges and corrects the prediction
        assert n_warm < n_cold
        total_cold += n_cold
        total_warm += n_warm
    print(f"total steps: cold {total_cold}, warm {total_warm} ({total_cold / total_warm:.2f}x)", flush=True)
    assert total_warm < 0.8 * total_cold


def test_prepared_prediction_has_no_staggered_velocity(predictions):
    _, pred = predictions
    sy = ((-1.0) ** np.arange(128))[:, None]
    sx = ((-1.0) ** np.arange(128))[None, :]
    for pf in pred:
        assert abs(np.mean(pf[1] * sy)) < 1e-6 and abs(np.mean(pf[0] * sx)) < 1e-6


def test_diverging_warm_start_falls_back_to_cold(predictions):
    """A prediction that makes the LB iteration diverge (a velocity far beyond
    the lattice's range) is caught by the residual kernel and that cavity is
    solved from rest instead; the other cavity keeps its warm start."""
    pds, pred = predictions
    cases = [W.ddc_case(pd) for pd in pds[:2]]
    bad = np.array(pred[:2])
    bad[1, 0] += 50.0  # u / u_lat: 5 lattice units
    out, flds = SS.solve_path(cases, bad, max_steps=1_500_000, log=print)
    assert out["fallback"] == [1]
    assert out["status"] == [lb.LBB_CONVERGED, lb.LBB_CONVERGED]
    cold = lb.Solver(*cases[1])
    cold.solve_steady(1e-8, 1000, 3_000_000)
    assert rel(flds[1], fields(cold)) < 1e-5


