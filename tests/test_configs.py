"""The named configurations (paper_2101_03055_amd/configs/*.json) load, build
records the library accepts, and carry the parameters their descriptions
state."""
import numpy as np
import pytest

from paper_2101_03055_amd import lb, workloads as W


def test_every_config_loads_and_validates():
    names = W.config_names()
    assert len(names) == 5
    for name in names:
        cfg, cases = W.load_config(name)
        assert cfg["description"] and cases
        if cfg["workload"] == "sweep_case":
            assert len(cases) == 200 and all(c["L"] == 128 for c in cases)
            continue
        for wl, phi0, u0, p0 in cases[:8]:
            for storage in cfg["run"]["storage"]:
                p = lb.params_from_workload(wl, storage, cfg["run"].get("phi_ref"), 100.0)
                assert lb.lb_workspace_bytes(p) > 0, (name, storage)
            assert np.isfinite(phi0).all() and np.isfinite(u0).all()


def test_stated_parameters():
    _, [(wl, phi0, *_)] = W.load_config("taylor_green_blobs_64")
    assert (wl["nx"], wl["ny"], wl["tau_f"]) == (64, 64, 0.8) and phi0.shape == (2, 64, 64)
    _, [(wl, *_)] = W.load_config("chemotaxis_plume_512x256")
    assert (wl["nx"], wl["ny"]) == (512, 256)
    assert abs(wl["tau_f"] - 1.4375) < 1e-12 and abs(0.5 + 3 * wl["D"][0][0] - 0.501875) < 1e-12
    _, [(wl, *_)] = W.load_config("ddc_cavity_256")
    assert (wl["nx"], wl["ny"]) == (256, 256) and abs(wl["tau_f"] - 0.6023) < 5e-5
    _, cases = W.load_config("ddc_sweep_256_cavities")
    sides = sorted({c[0]["nx"] for c in cases})
    assert len(cases) == 256 and sides[0] >= 64 and sides[-1] <= 256 and all(s % 32 == 0 for s in sides)
