"""Two steps per launch (fused_steps = 2, temporal blocking through LDS)
against the one-step AA-pattern path and the oracle.

Both paths apply the same per-node update to the same values, so they agree
to rounding (the compiler may contract the same expressions differently in
the two kernels); mixed odd/even step counts exercise the hand-over between
the AA layouts and the two-array layout."""
import numpy as np
import pytest

from paper_2101_03055_amd import lb, workloads as W
from test_gpu_parity import BC_CASES, plane_errors

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("case", sorted(BC_CASES))
@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_two_step_matches_one_step(case, storage):
    fb, sb = BC_CASES[case]
    wl, phi0, u0, p0 = W.random_case(131, 37, m=2, seed=17, fluid_bc=fb, scalar_bc=sb, force=True, source=True)
    ref = [1.0, 1.0]
    a = lb.Solver(wl, phi0, u0, p0, storage=storage, phi_ref=ref)
    b = lb.Solver(wl, phi0, u0, p0, storage=storage, phi_ref=ref, fused_steps=2)
    for n in (1, 4, 3, 6, 0, 9):
        a.step(n)
        b.step(n)
    assert a.t == b.t == 23
    fa, ha = a.populations()
    fb_, hb = b.populations()
    tol = 1e-13 if storage == "f64" else 1e-6
    e = max(plane_errors(fb_, fa), plane_errors(hb, ha))
    print(f"{case} {storage}: two-step vs one-step {e:.2e}", flush=True)
    assert e <= tol


def test_two_step_matches_oracle(oracle_mod):
    for name in ("cavity_noslip_dirichlet", "channel_freeslip_top"):
        fb, sb = BC_CASES[name]
        wl, phi0, u0, p0 = W.random_case(67, 45, m=2, seed=7, fluid_bc=fb, scalar_bc=sb, force=True)
        o = oracle_mod.Oracle(wl, phi0, u0, p0)
        g = lb.Solver(wl, phi0, u0, p0, fused_steps=2)
        o.step(200)
        g.step(200)
        f, h = g.populations()
        assert plane_errors(f, o.f) <= 1e-11 and plane_errors(h, o.h) <= 1e-11


def test_two_step_plume_full_size(oracle_mod):
    wl, phi0, u0, p0 = W.chemotaxis_plume()
    o = oracle_mod.Oracle(wl, phi0, u0, p0)
    g = lb.Solver(wl, phi0, u0, p0, fused_steps=2)
    o.step(100)
    g.step(100)
    f, h = g.populations()
    assert plane_errors(f, o.f) <= 1e-11 and plane_errors(h, o.h) <= 1e-11


def test_two_step_small_periodic_domain():
    """Domains narrower than the tile ring wrap several times in LDS."""
    wl, phi0, u0, p0 = W.random_case(5, 3, m=1, seed=2)
    a = lb.Solver(wl, phi0, u0, p0)
    b = lb.Solver(wl, phi0, u0, p0, fused_steps=2)
    a.step(40)
    b.step(40)
    fa, ha = a.populations()
    fb, hb = b.populations()
    assert max(plane_errors(fb, fa), plane_errors(hb, ha)) <= 1e-13
