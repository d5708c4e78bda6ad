"""Batched sweep (lbb_*): many cavities of uneven size in one launch per step.

The batched kernel runs the same per-node update as the single-domain kernel,
so every cavity of a batch must match its own single-domain run bit for bit
(and hence the oracle), independently of the tile shape, of the other
cavities, and of when it is retired.
"""
import numpy as np
import pytest

from paper_2101_03055_amd import lb, workloads as W

pytestmark = pytest.mark.gpu


def mixed_cases():
    cases = [W.ddc(64, Ra=1e4, Pr=0.71, Le=2.0, Nc=1.0, Sr=0.1, Df=0.1),
             W.ddc(96, Ra=1e5, Pr=0.71, Le=3.0, Nc=-0.5, Sr=0.2, Df=0.05),
             W.random_case(70, 33, seed=41, fluid_bc=["noslip", "noslip", "noslip", "freeslip"],
                           scalar_bc=[["dirichlet"] * 2, ["noflux"] * 2, ["noflux"] * 2, ["dirichlet"] * 2]),
             W.random_case(50, 61, seed=42, source=True, fluid_bc=["periodic", "periodic", "noslip", "noslip"],
                           scalar_bc=[["periodic"] * 2, ["periodic"] * 2, ["noflux"] * 2, ["dirichlet"] * 2]),
             W.ddc(32, Ra=1e3, Pr=0.71, Le=1.5, Nc=0.5, Sr=0.0, Df=0.3, A=2.0)]
    return cases


def single(case, steps, storage="f64", **kw):
    s = lb.Solver(*case, storage=storage, **kw)
    s.step(steps)
    return s.moments()


@pytest.mark.parametrize("tile", [(64, 4), (32, 8), (128, 1)])
def test_batch_equals_single_domain_bitwise(tile):
    cases = mixed_cases()
    b = lb.Batch(cases)
    lb.lbb_set_tile(b.handle, *tile)
    b.step(37)
    for i, c in enumerate(cases):
        got = b.moments(i)
        want = single(c, 37)
        for g, w in zip(got, want):
            assert np.array_equal(g, w), (tile, i)


def test_batch_f32_equals_single_domain_bitwise():
    cases = mixed_cases()
    ref = [0.5, 0.5]
    b = lb.Batch(cases, storage="f32", phi_ref=ref)
    b.step(24)
    for i, c in enumerate(cases):
        got = b.moments(i)
        want = single(c, 24, storage="f32", phi_ref=ref)
        for g, w in zip(got, want):
            assert np.array_equal(g, w), i


def test_batch_cavity_against_oracle(oracle_mod):
    cases = mixed_cases()
    b = lb.Batch(cases)
    b.step(200)
    for i in (1, 3):
        wl, phi0, u0, p0 = cases[i]
        o = oracle_mod.Oracle(wl, phi0, u0, p0)
        o.step(200)
        phi, u, _ = b.moments(i)
        po, uo, _ = o.moments()
        for a in range(2):
            assert np.abs(phi[a] - po[a]).max() / np.abs(po[a]).max() <= 1e-11
        for d in range(2):
            assert np.abs(u[d] - uo[d]).max() / np.abs(uo[d]).max() <= 1e-11


def test_run_retires_cavities_at_their_own_step():
    """After lbb_run every cavity equals a single-domain run of exactly the
    number of steps it took: retirement freezes the state."""
    cases = [W.ddc(32, Ra=1e3, Pr=0.71, Le=1.0, Nc=0.0, Sr=0.0, Df=0.0),
             W.ddc(48, Ra=1e4, Pr=0.71, Le=2.0, Nc=1.0, Sr=0.1, Df=0.1),
             W.ddc(64, Ra=3e4, Pr=0.71, Le=2.0, Nc=-0.5, Sr=0.2, Df=0.2)]
    b = lb.Batch(cases)
    steps, status, res = b.run(tol=1e-6, check_every=500, max_steps=400_000)
    print("batch run:", steps.tolist(), status.tolist(), res.max(axis=1).tolist(), flush=True)
    assert np.all(status == lb.LBB_CONVERGED)
    assert len(set(steps.tolist())) > 1
    assert np.all(res < 1e-6)
    for i, c in enumerate(cases):
        want = single(c, int(steps[i]))
        got = b.moments(i)
        for g, w in zip(got, want):
            assert np.array_equal(g, w), i


def test_divergence_is_isolated():
    good = W.ddc(32, Ra=1e3, Pr=0.71, Le=1.0, Nc=0.0, Sr=0.0, Df=0.0)
    bad = W.ddc(40, Ra=1e3, Pr=0.71, Le=1.0, Nc=0.0, Sr=0.0, Df=0.0)
    bad[0]["F0"] = [1e300, 1e300]
    b = lb.Batch([good, bad])
    steps, status, _ = b.run(tol=1e-6, check_every=200, max_steps=200_000)
    assert status.tolist() == [lb.LBB_CONVERGED, lb.LBB_DIVERGED]
    assert steps[1] == 200


def test_autotune_picks_a_supported_tile_and_keeps_results():
    cases = mixed_cases()
    b = lb.Batch(cases)
    tx, ty, us = b.autotune(10)
    assert (tx, ty) in [(32, 4), (32, 8), (64, 2), (64, 4), (128, 1), (128, 2), (256, 1)]
    assert us > 0
    shapes = [b.cavity_tile(i) for i in range(len(cases))]
    assert all(sx * sy == tx * ty for sx, sy in shapes), shapes
    taken = b.time(0)[0]
    # 7 shapes for all cavities, then per width a fresh timing and the other shapes of the
    # same workgroup size, each 10 + 2 steps
    assert taken >= 7 * (10 + 2) and taken % 12 == 0
    b.step(6)
    for i, c in enumerate(cases):
        got = b.moments(i)
        want = single(c, taken + 6)
        for g, w in zip(got, want):
            assert np.array_equal(g, w), i


def test_per_cavity_tiles_keep_results():
    """Each cavity with its own tile shape (all of one workgroup size): every cavity
    still matches its single-domain run bit for bit; a shape of another size is refused."""
    cases = mixed_cases()
    b = lb.Batch(cases)
    lb.lbb_set_tile(b.handle, 64, 4)
    for i, sh in enumerate([(256, 1), (32, 8), (128, 2), (64, 4), (256, 1)]):
        lb.lbb_set_cavity_tile(b.handle, i, *sh)
        assert b.cavity_tile(i) == sh
    with pytest.raises(lb.LBError):
        lb.lbb_set_cavity_tile(b.handle, 0, 64, 2)
    b.step(41)
    for i, c in enumerate(cases):
        got = b.moments(i)
        want = single(c, 41)
        for g, w in zip(got, want):
            assert np.array_equal(g, w), i


def test_copy_cavity_between_batches():
    """FP32 batch -> FP64 batch (exact widening), then both continue like a
    single-domain FP64 run started from the copied state."""
    cases = mixed_cases()[:3]
    a = lb.Batch(cases, storage="f32", phi_ref=[0.5, 0.5])
    a.step(21)  # odd: the source cavities are in the even-step layout
    b = lb.Batch(cases, storage="f64")
    for i in range(3):
        lb.lbb_copy_cavity(b.handle, i, a.handle, i)
    for i in range(3):
        assert b.time(i)[0] == 21
        ga, gb = a.moments(i), b.moments(i)
        for x, y in zip(ga[:2], gb[:2]):
            assert np.abs(x - y).max() <= 1e-6 * max(1.0, np.abs(y).max())
    # the copied FP64 cavity evolves exactly like a single FP64 run loaded with the same populations
    s = lb.Solver(*cases[1], storage="f64")
    sa = lb.Solver(*cases[1], storage="f32", phi_ref=[0.5, 0.5])
    sa.step(21)
    lb.lb_copy_state(s.handle, sa.handle)
    b.step(10)
    s.step(10)
    for x, y in zip(b.moments(1), s.moments()):
        assert np.array_equal(x, y)


def test_copy_cavity_rejects_mismatched_parameters():
    cases = mixed_cases()
    a = lb.Batch(cases[:2])
    b = lb.Batch(cases[:2])
    with pytest.raises(lb.LBError):
        lb.lbb_copy_cavity(b.handle, 0, a.handle, 1)


def test_full_sweep_sampled_cavities(oracle_mod):
    """The 256-cavity sweep at its full size (8.0 M nodes, sides 64..256), as
    benchmarked: FP32 after autotuning, every sampled cavity bitwise equal to
    a single-domain FP32 run; and FP64 on the same batch, the smallest, the
    largest and a middle cavity against the oracle after 300 steps (both
    parities visited) at 1e-11."""
    pds = W.sweep_params(256, seed=4)
    cases = [W.ddc_case(pd) for pd in pds]
    sizes = [c[0]["nx"] * c[0]["ny"] for c in cases]
    pick = sorted({int(np.argmin(sizes)), int(np.argmax(sizes)), len(cases) // 2})

    b32 = lb.Batch(cases, storage="f32", phi_ref=[0.5, 0.5])
    b32.autotune(4)
    b32.step(301 - b32.time(0)[0])
    for i in pick:
        s = lb.Solver(*cases[i], storage="f32", phi_ref=[0.5, 0.5])
        s.step(301)
        phi_b, u_b, _ = b32.moments(i)
        phi_s, u_s, _ = s.moments()
        assert np.array_equal(phi_b, phi_s) and np.array_equal(u_b, u_s), f"cavity {i}"
        s.close()
    b32.close()

    b64 = lb.Batch(cases, storage="f64")
    b64.step(300)
    for i in pick:
        wl, phi0, u0, p0 = cases[i]
        o = oracle_mod.Oracle(wl, phi0, u0, p0)
        o.step(300)
        phi, u, _ = b64.moments(i)
        po, uo, _ = o.moments()
        e = max(max(np.abs(phi[a] - po[a]).max() / np.abs(po[a]).max() for a in range(2)),
                max(np.abs(u[d] - uo[d]).max() / np.abs(uo[d]).max() for d in range(2)))
        print(f"sweep cavity {i} ({wl['nx']}x{wl['ny']}): FP64 vs oracle {e:.2e}", flush=True)
        assert e <= 1e-11
