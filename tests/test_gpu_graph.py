"""lb_step replays a prebuilt graph of 64 single-step launches for long runs.
Every replay must equal the plain launch path bit for bit, with the program's
own eager work and synchronisations between replays, across a tile change
(graph rebuilt) and from either AA parity.  FP16 included: a replayed launch
takes its stochastic-rounding salt from the step count the host sets before
the replay, so the dither equals that of the plain launches."""
import numpy as np
import pytest

from paper_2101_03055_amd import lb, workloads as W

pytestmark = pytest.mark.gpu


def eager(s, n):
    for _ in range(n):
        s.step(1)  # below the graph threshold: one launch per call


F16 = {"storage": "f16", "phi_ref": [1.0, 1.0], "fp16_scale": 100.0, "fp16_scale_h": 1000.0}


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
@pytest.mark.parametrize("kind", ["walls", "chemotaxis"])
def test_graph_replays_equal_plain_launches(storage, kind):
    if kind == "walls":
        case = W.random_case(70, 45, seed=61, fluid_bc=["noslip", "noslip", "freeslip", "noslip"],
                             scalar_bc=[["dirichlet"] * 2, ["noflux"] * 2, ["dirichlet"] * 2, ["noflux"] * 2])
    else:
        case = W.random_case(64, 40, seed=62, model="chemotaxis", fluid_bc=["periodic", "periodic", "noslip", "freeslip"],
                             scalar_bc=[["periodic"] * 2, ["periodic"] * 2, ["noflux"] * 2, ["noflux", "dirichlet"]])
    kw = {"f32": {"storage": "f32", "phi_ref": [1.0, 1.0]}, "f16": F16}.get(storage, {})
    g = lb.Solver(*case, **kw)
    e = lb.Solver(*case, **kw)
    for n, tile in ((64, None), (65, None), (130, (128, 1)), (64, (64, 2)), (193, None)):
        if tile:
            lb.lb_set_tile(g.handle, *tile)
            lb.lb_set_tile(e.handle, *tile)
        g.step(n)
        eager(e, n)
        assert g.t == e.t
        for x, y in zip(g.moments(), e.moments()):
            assert np.all(np.isfinite(x)) and np.array_equal(x, y), (n, tile)
        g.residual()
        e.residual()
    fg, hg = lb.lb_populations(g.handle, g.m, g.ny, g.nx)
    fe, he = lb.lb_populations(e.handle, e.m, e.ny, e.nx)
    assert np.array_equal(fg, fe) and np.array_equal(hg, he)


def test_batched_graph_replays_equal_plain_launches():
    cases = [W.ddc(48, Ra=1e4, Pr=0.71, Le=2.0, Nc=1.0, Sr=0.1, Df=0.1),
             W.random_case(50, 61, seed=42, source=True, fluid_bc=["periodic", "periodic", "noslip", "noslip"],
                           scalar_bc=[["periodic"] * 2, ["periodic"] * 2, ["noflux"] * 2, ["dirichlet"] * 2]),
             W.ddc(32, Ra=1e3, Pr=0.71, Le=1.5, Nc=0.5, Sr=0.0, Df=0.3, A=2.0)]
    for storage in ("f64", "f32", "f16"):
        kw = {"f32": {"storage": "f32", "phi_ref": [0.5, 0.5]},
              "f16": {"storage": "f16", "phi_ref": [0.5, 0.5], "fp16_scale": 1e3, "fp16_scale_h": 1e4}}.get(storage, {"storage": storage})
        g = lb.Batch(cases, **kw)
        e = lb.Batch(cases, **kw)
        for n in (64, 131, 70):
            g.step(n)
            for _ in range(n):
                e.step(1)
            for i in range(len(cases)):
                for x, y in zip(g.moments(i), e.moments(i)):
                    assert np.all(np.isfinite(x)) and np.array_equal(x, y), (storage, n, i)


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_no_fluid_graph_replays_equal_plain_launches(storage):
    """The no-fluid model (prescribed flow) replays its step graph the same way."""
    case = W.cde_case(67, 45, m=2, seed=5, walls=True, source=True)
    kw = {"storage": "f32", "phi_ref": [1.0, 1.0]} if storage == "f32" else {}
    g = lb.Solver(*case, **kw)
    e = lb.Solver(*case, **kw)
    for n, tile in ((64, None), (65, None), (130, (64, 2)), (193, None)):
        if tile:
            lb.lb_set_tile(g.handle, *tile)
            lb.lb_set_tile(e.handle, *tile)
        g.step(n)
        eager(e, n)
        assert g.t == e.t
        for x, y in zip(g.moments(), e.moments()):
            assert np.all(np.isfinite(x)) and np.array_equal(x, y), (n, tile)
        g.residual()
        e.residual()
