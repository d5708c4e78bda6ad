"""lb_residual_noalloc (the residual entry point that allocates nothing: its
reduction scratch is a library-held device array) against lb_residual: two
identical solvers, one read through each entry point, must report bitwise
equal residuals -- the same kernels in the same order over the same state --
on a first grid and then on a smaller one, so that the second call finds the
array holding the first call's larger contents."""
import numpy as np
import pytest

from paper_2101_03055_amd import lb, workloads as W

pytestmark = pytest.mark.gpu


def pair(nx, ny, seed, storage="f64", model_kw=None):
    wl, phi0, u0, p0 = W.random_case(nx, ny, m=2, seed=seed, fluid_bc=["noslip"] * 4,
                                     scalar_bc=[["dirichlet", "noflux"]] * 4, source=True)
    a = lb.Solver(wl, phi0, u0, p0, storage=storage, phi_ref=[1.0, 1.0])
    b = lb.Solver(wl, phi0, u0, p0, storage=storage, phi_ref=[1.0, 1.0])
    return a, b


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_noalloc_residual_equals_residual_then_smaller_grid(storage):
    for (nx, ny, seed) in [(300, 211, 1), (37, 23, 2)]:   # the second grid is smaller
        a, b = pair(nx, ny, seed, storage)
        r0, s0 = lb.lb_residual(a.handle, 2)
        q0, t0 = lb.lb_residual_noalloc(b.handle, 2)
        assert s0 == t0 == lb.LB_OK and np.all(np.isinf(r0)) and np.all(np.isinf(q0))
        for k in (7, 50):
            a.step(k)
            b.step(k)
            r, s = lb.lb_residual(a.handle, 2)
            q, t = lb.lb_residual_noalloc(b.handle, 2)
            print(f"{nx}x{ny} {storage} after {k} more steps: {r} vs {q}", flush=True)
            assert s == t == lb.LB_OK
            assert np.array_equal(r, q)
            assert np.all(r > 0)


def test_noalloc_residual_no_fluid_model():
    wl, phi0, u0, p0 = W.cde_case(96, 64, m=2, seed=3)
    a = lb.Solver(wl, phi0, u0, p0, storage="f64")
    b = lb.Solver(wl, phi0, u0, p0, storage="f64")
    for k in (0, 9, 40):
        a.step(k)
        b.step(k)
        r, s = lb.lb_residual(a.handle, 2)
        q, t = lb.lb_residual_noalloc(b.handle, 2)
        assert s == t and (np.array_equal(r, q))
