"""Variants of the model beyond the settings of the paper's experiments: a
general lambda in the scalar equilibrium (Eq. feq-phi with Eq. omega-D) and the
varphi term of the discrete force (Eq. force, pressure of appendix A).  The HIP
path against the oracle on the same seeded inputs, through every launch path
(single steps, replayed step graphs, two-step launches, the batched kernel and
the no-fluid model)."""
import numpy as np
import pytest

from paper_2101_03055_amd import lb, workloads as W
from test_gpu_parity import BC_CASES, moment_errors, plane_errors, pop_errors

pytestmark = pytest.mark.gpu
TOL64 = 1e-11

LAM2 = [[0.6, 0.3], [-0.1, 1.2]]
LAM3 = [[0.9, 0.1, 0.0], [-0.1, 1.1, 0.2], [0.05, 0.0, 0.8]]


def variant_case(name, m=2, seed=7, lam=None, varphi=0.0, source=True):
    fb, sb = BC_CASES[name]
    if m != 2:
        sb = [[r[0]] * m for r in sb]
    wl, phi0, u0, p0 = W.random_case(67, 45, m=m, seed=seed, fluid_bc=fb, scalar_bc=sb, force=True, source=source)
    if lam is not None:
        wl["lam"] = lam
    wl["varphi"] = varphi
    return wl, phi0, u0, p0


def run_pair(oracle_mod, case, steps, storage="f64", **kw):
    wl, phi0, u0, p0 = case
    o = oracle_mod.Oracle(wl, phi0, u0, p0)
    g = lb.Solver(wl, phi0, u0, p0, storage=storage, **kw)
    o.step(steps)
    g.step(steps)
    return o, g


@pytest.mark.parametrize("name", sorted(BC_CASES))
@pytest.mark.parametrize("steps", [37, 200])
def test_lambda_matches_oracle(oracle_mod, name, steps):
    o, g = run_pair(oracle_mod, variant_case(name, lam=LAM2), steps)
    ef, eh = pop_errors(o, g)
    print(f"lambda {name} {steps}: f {ef:.2e} h {eh:.2e}", flush=True)
    assert ef <= TOL64 and eh <= TOL64
    assert moment_errors(o, g) <= TOL64


def test_lambda_three_species(oracle_mod):
    o, g = run_pair(oracle_mod, variant_case("cavity_noslip_dirichlet", m=3, seed=9, lam=LAM3), 151)
    ef, eh = pop_errors(o, g)
    assert ef <= TOL64 and eh <= TOL64


@pytest.mark.parametrize("name", sorted(BC_CASES))
@pytest.mark.parametrize("varphi", [1.0, 0.5])
def test_varphi_matches_oracle(oracle_mod, name, varphi):
    o, g = run_pair(oracle_mod, variant_case(name, varphi=varphi), 200)
    ef, eh = pop_errors(o, g)
    em = moment_errors(o, g)  # includes the pressure with its varphi correction
    print(f"varphi {varphi} {name}: f {ef:.2e} h {eh:.2e} moments {em:.2e}", flush=True)
    assert ef <= TOL64 and eh <= TOL64 and em <= TOL64


def test_varphi_changes_the_result(oracle_mod):
    """The varphi terms are live: the run differs from varphi = 0 by far more
    than the parity tolerance."""
    a = lb.Solver(*variant_case("cavity_noslip_dirichlet", varphi=1.0))
    b = lb.Solver(*variant_case("cavity_noslip_dirichlet", varphi=0.0))
    a.step(200)
    b.step(200)
    _, ha = a.populations()
    _, hb = b.populations()
    assert plane_errors(ha, hb) > 1e-8


def test_both_variants_two_step_launches(oracle_mod):
    case = variant_case("channel_freeslip_top", lam=LAM2, varphi=1.0)
    o, g = run_pair(oracle_mod, case, 200, fused_steps=2)
    ef, eh = pop_errors(o, g)
    assert ef <= TOL64 and eh <= TOL64


def test_both_variants_fp32(oracle_mod):
    case = variant_case("cavity_noslip_dirichlet", lam=LAM2, varphi=1.0)
    o, g = run_pair(oracle_mod, case, 500, storage="f32", phi_ref=[1.0, 1.0])
    phi, u, p = g.moments()
    po, uo, _ = o.moments()
    ephi = max(np.abs(phi[a] - po[a]).max() / np.abs(po[a]).max() for a in range(2))
    eu = max(np.abs(u[d] - uo[d]).max() / np.abs(uo[d]).max() for d in range(2))
    print(f"fp32 lambda+varphi: phi {ephi:.2e} u {eu:.2e}", flush=True)
    assert ephi <= 2e-6 and eu <= 2e-4


def test_batch_with_variants_equals_single_domain_bitwise():
    cases = [variant_case("cavity_noslip_dirichlet", lam=LAM2, varphi=1.0),
             variant_case("channel_freeslip_top", seed=8, varphi=0.5),
             variant_case("periodic_y_walls_x", seed=9, lam=LAM2)]
    b = lb.Batch(cases)
    b.step(37)
    for i, c in enumerate(cases):
        s = lb.Solver(*c)
        s.step(37)
        for got, want in zip(b.moments(i), s.moments()):
            assert np.array_equal(got, want), i


@pytest.mark.parametrize("walls", [False, True])
def test_no_fluid_model_with_lambda(oracle_mod, walls):
    wl, phi0, u0, p0 = W.cde_case(67, 45, m=2, seed=5, walls=walls, source=True)
    wl["lam"] = LAM2
    o = oracle_mod.Oracle(wl, phi0, u0, p0)
    g = lb.Solver(wl, phi0, u0, p0)
    o.step(151)
    g.step(151)
    f, _ = g.populations()
    ef = max(np.abs(f[a, i] - o.f[a, i]).max() / np.abs(o.f[a, i]).max() for a in range(2) for i in range(5))
    print(f"no-fluid lambda walls {walls}: f {ef:.2e}", flush=True)
    assert ef <= TOL64


# ---- gamma of D-bar (Eq. evolution12) ----------------------------------------
GAM = [1.7, -0.9, 0.6]


def gamma_case(name, m=2, seed=7, model="linear"):
    fb, sb = BC_CASES[name]
    if m != 2:
        sb = [[r[0]] * m for r in sb]
    wl, phi0, u0, p0 = W.random_case(67, 45, m=m, seed=seed, fluid_bc=fb, scalar_bc=sb, force=True, source=True,
                                     model=model, amp=0.2)
    wl["K"] = (np.asarray(wl["K"]) * 20).tolist()   # sources strong enough for the gamma term to matter
    wl["gamma_s"] = GAM[:m]
    return wl, phi0, u0, p0


@pytest.mark.parametrize("name", sorted(BC_CASES))
def test_gamma_matches_oracle(oracle_mod, name):
    """Through single launches of both parities and replayed step graphs (the
    two source buffers alternate): 1, 2, 37, 130 steps."""
    wl, phi0, u0, p0 = gamma_case(name)
    o = oracle_mod.Oracle(wl, phi0, u0, p0)
    g = lb.Solver(wl, phi0, u0, p0)
    for n in (1, 2, 37, 130):
        o.step(n)
        g.step(n)
        ef, eh = pop_errors(o, g)
        print(f"gamma {name} t = {g.t}: f {ef:.2e} h {eh:.2e}", flush=True)
        assert ef <= TOL64 and eh <= TOL64
    assert moment_errors(o, g) <= TOL64


def test_gamma_three_species_and_chemotaxis(oracle_mod):
    for case in (gamma_case("cavity_noslip_dirichlet", m=3, seed=9),
                 gamma_case("channel_freeslip_top", seed=11, model="chemotaxis")):
        o = oracle_mod.Oracle(*case)
        g = lb.Solver(*case)
        o.step(151)
        g.step(151)
        ef, eh = pop_errors(o, g)
        print(f"gamma {case[0]['model']} m = {case[0]['m']}: f {ef:.2e} h {eh:.2e}", flush=True)
        assert ef <= TOL64 and eh <= TOL64


def test_gamma_changes_the_result():
    wl, phi0, u0, p0 = gamma_case("periodic_y_walls_x")
    a = lb.Solver(wl, phi0, u0, p0)
    b = lb.Solver(dict(wl, gamma_s=[0.0, 0.0]), phi0, u0, p0)
    a.step(100)
    b.step(100)
    fa, _ = a.populations()
    fb, _ = b.populations()
    assert plane_errors(fa, fb) > 1e-9


def test_gamma_save_load_and_fp32(oracle_mod):
    """Checkpoints at odd and even steps resume bit for bit (the current source
    buffer alternates); FP32 storage stays within its usual error."""
    case = gamma_case("cavity_noslip_dirichlet")
    for k in (41, 64):
        a = lb.Solver(*case)
        a.step(k)
        blob = lb.lb_save(a.handle)
        a.step(99)
        fa, ha = a.populations()
        b = lb.Solver(*case)
        b.step(3)                     # a different buffer parity before the load
        lb.lb_load(b.handle, blob)
        b.step(99)
        fb, hb = b.populations()
        assert np.array_equal(fa, fb) and np.array_equal(ha, hb), k
    o = oracle_mod.Oracle(*case)
    g = lb.Solver(*case, storage="f32", phi_ref=[1.0, 1.0])
    o.step(500)
    g.step(500)
    phi, u, _ = g.moments()
    po, uo, _ = o.moments()
    ephi = max(np.abs(phi[a] - po[a]).max() / np.abs(po[a]).max() for a in range(2))
    print(f"gamma fp32: phi {ephi:.2e}", flush=True)
    assert ephi <= 2e-6
