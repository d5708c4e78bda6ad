"""Case 1 of the model (no fluid, prescribed velocity, LB_MODEL_CDE): the GPU
path against the oracle on the same seeded inputs."""
import numpy as np
import pytest

from paper_2101_03055_amd import lb, workloads as W

pytestmark = pytest.mark.gpu
TOL64 = 1e-11


def errors(o, g):
    f, hp = g.populations()
    assert not hp.any()  # no fluid populations
    ef = max(np.abs(f[a, i] - o.f[a, i]).max() / np.abs(o.f[a, i]).max()
             for a in range(f.shape[0]) for i in range(5))
    phi, u, p = g.moments()
    po, uo, _ = o.moments()
    em = max(np.abs(phi[a] - po[a]).max() / np.abs(po[a]).max() for a in range(phi.shape[0]))
    return ef, em, u, uo, p


@pytest.mark.parametrize("steps", [150, 151])
@pytest.mark.parametrize("walls,source,m", [(False, False, 2), (False, True, 3), (True, False, 2), (True, True, 1)])
def test_matches_oracle_fp64(oracle_mod, steps, walls, source, m):
    wl, phi0, u0, p0 = W.cde_case(67, 45, m=m, seed=3 + m, walls=walls, source=source)
    o = oracle_mod.Oracle(wl, phi0, u0, p0)
    g = lb.Solver(wl, phi0, u0, p0)
    o.step(steps)
    g.step(steps)
    ef, em, u, uo, p = errors(o, g)
    print(f"walls {walls} source {source} m {m} steps {steps}: f {ef:.2e} phi {em:.2e}", flush=True)
    assert ef <= TOL64 and em <= TOL64
    assert np.array_equal(u, u0) and np.array_equal(uo, u0) and not p.any()


def test_fp32_close_to_oracle(oracle_mod):
    wl, phi0, u0, p0 = W.cde_case(64, 48, m=2, seed=9, walls=True, source=True)
    o = oracle_mod.Oracle(wl, phi0, u0, p0)
    g = lb.Solver(wl, phi0, u0, p0, storage="f32", phi_ref=[1.0, 1.0])
    o.step(500)
    g.step(500)
    phi, _, _ = g.moments()
    po, _, _ = o.moments()
    err = max(np.abs(phi[a] - po[a]).max() / np.abs(po[a]).max() for a in range(2))
    print(f"fp32 phi error {err:.2e}", flush=True)
    assert err <= 2e-6


def test_mass_residual_and_resume():
    wl, phi0, u0, p0 = W.cde_case(48, 40, m=2, seed=11)
    g = lb.Solver(wl, phi0, u0, p0)
    m0, _ = g.mass()
    g.step(300)
    m1, _ = g.mass()
    assert np.abs(m1[:2] - m0[:2]).max() <= 1e-12 * np.abs(m0[:2]).max()
    assert m1[2] == 0.0
    g.residual()
    g.step(100)
    r, _ = g.residual()
    assert r[0] == 0.0 and r[1] == 0.0 and np.all(np.isfinite(r)) and r[2:].max() > 0
    blob = lb.lb_save(g.handle)
    g.step(37)
    want = g.moments()
    h = lb.Solver(wl, phi0, u0, p0)
    lb.lb_load(h.handle, blob)
    h.step(37)
    for x, y in zip(h.moments(), want):
        assert np.array_equal(x, y)


def test_unavailable_calls_are_rejected():
    wl, phi0, u0, p0 = W.cde_case(32, 32, m=2, seed=1, walls=True)
    g = lb.Solver(wl, phi0, u0, p0)
    with pytest.raises(lb.LBError):
        lb.lb_wall_flux(g.handle, 0, 2)
    other = lb.Solver(wl, phi0, u0, p0)
    with pytest.raises(lb.LBError):
        lb.lb_copy_state(other.handle, g.handle)
