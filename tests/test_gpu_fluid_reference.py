"""The fluid reference pressure per row (lb_fluid_reference): the stored fluid
populations become departures from the rest equilibrium at the row's reference
pressure, and values that stream between rows change reference on the way.

* In FP64 the reference changes nothing but rounding: runs with and without it,
  switched on at either AA parity, refreshed, replayed through the step graphs
  and switched off again, agree to 1e-12 on every wall rule of the fluid (no
  slip, free slip on x and on y walls, periodic rows that wrap the reference).
* lb_save / lb_load keep the reference (a continued run is bitwise equal), and
  lb_copy_state hands the absolute values to a handle without one.
* Not for the no-fluid model or two steps per launch.
"""
import numpy as np
import pytest

from paper_2101_03055_amd import lb, workloads as W

pytestmark = pytest.mark.gpu

CASES = {
    "walls": (["freeslip", "noslip", "noslip", "noslip"],
              [["noflux", "dirichlet"], ["dirichlet", "noflux"], ["noflux", "noflux"], ["dirichlet", "dirichlet"]]),
    "periodic_rows": (["noslip", "freeslip", "periodic", "periodic"],
                      [["noflux", "noflux"], ["dirichlet", "noflux"], ["periodic", "periodic"], ["periodic", "periodic"]]),
    "freeslip_y": (["periodic", "periodic", "freeslip", "freeslip"],
                   [["periodic", "periodic"], ["periodic", "periodic"], ["noflux", "noflux"], ["noflux", "dirichlet"]]),
}


def make(name, storage="f64", **kw):
    fbc, sbc = CASES[name]
    wl, phi0, u0, p0 = W.random_case(96, 70, m=2, seed=11, fluid_bc=fbc, scalar_bc=sbc)
    # a vertical body force, so that the rows carry a hydrostatic pressure gradient
    wl["F0"] = [0.0, -2e-5]
    return lb.Solver(wl, phi0, u0, p0, storage=storage, **kw)


def compare(a, b, label):
    fa, ha = a.populations()
    fb, hb = b.populations()
    eh = float(np.abs(ha - hb).max() / np.abs(ha).max())
    ef = float(np.abs(fa - fb).max() / np.abs(fa).max())
    pa, ua, qa = a.moments()
    pb, ub, qb = b.moments()
    ep = float(np.abs(qa - qb).max() / np.abs(qa).max())
    eu = float(np.abs(ua - ub).max() / np.abs(ua).max())
    print(f"{label}: h {eh:.1e} f {ef:.1e} p {ep:.1e} u {eu:.1e}", flush=True)
    assert max(eh, ef) < 1e-12 and ep < 1e-11 and eu < 1e-11, label


@pytest.mark.parametrize("name", sorted(CASES))
def test_reference_changes_nothing_in_fp64(name):
    a, b = make(name), make(name)
    for s in (a, b):
        s.step(201)                  # odd: the reference is first set on the layout left by an even step
    b.fluid_reference(1)
    compare(a, b, f"{name}, reference set")
    for s in (a, b):
        s.step(150)
    b.fluid_reference(1)             # refreshed, again at parity 1
    for s in (a, b):
        s.step(200)                  # replayed step graphs (64 launches each) and single launches
    compare(a, b, f"{name}, 551 steps")
    b.fluid_reference(0)
    for s in (a, b):
        s.step(11)
    compare(a, b, f"{name}, reference dropped")


def test_save_load_and_copy_keep_the_absolute_state():
    a = make("walls", storage="f32", phi_ref=[1.0, 1.0])
    a.step(300)
    a.fluid_reference(1)
    a.step(101)
    blob = lb.lb_save(a.handle)
    a.step(257)
    b = make("walls", storage="f32", phi_ref=[1.0, 1.0])
    lb.lb_load(b.handle, blob)
    b.step(257)
    fa, ha = a.populations()
    fb, hb = b.populations()
    assert np.array_equal(fa, fb) and np.array_equal(ha, hb)
    # into FP64 storage without a reference: the same absolute populations
    c = make("walls", storage="f64")
    lb.lb_copy_state(c.handle, a.handle)
    fc, hc = c.populations()
    assert np.array_equal(fa, fc) and np.array_equal(ha, hc)


def test_reference_is_rejected_where_it_does_not_apply():
    wl, phi0, u0, p0 = W.cde_case(64, 48, m=2, seed=1)
    s = lb.Solver(wl, phi0, u0, p0)
    with pytest.raises(lb.LBError):
        s.fluid_reference(1)
    t = make("walls", fused_steps=2)
    with pytest.raises(lb.LBError):
        t.fluid_reference(1)
    u = make("walls")
    with pytest.raises(lb.LBError):
        lb.lb_fluid_reference(u.handle, 2)
