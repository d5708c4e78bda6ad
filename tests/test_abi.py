"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/lb.h declares, its record matches the binding, and
lb_init / lb_workspace_bytes reject bad inputs before touching a device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2101_03055_amd import lb, workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared(header):
    with open(os.path.join(ROOT, "include", header)) as fh:
        text = fh.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b((?:lb|sg|lbb|lb3)_[a-z_0-9]+)\s*\(", text)))


@pytest.mark.parametrize("header", ["lb.h", "sg.h", "lb3.h"])
def test_library_exports_every_declared_symbol(header):
    L = lb.lib()
    names = declared(header)
    assert len(names) >= 10
    for name in names:
        assert hasattr(L, name), name


def test_surrogate_host_queries():
    from paper_2101_03055_amd import sg
    packed, real = sg.param_count()
    assert 200_000 < real < 300_000 and packed > real
    assert sg.layer_info(0) == (15, 64, 32, 64) and sg.layer_info(5) == (64, 4, 64, 64)


def test_params_record_matches():
    assert lb.lib().lb_params_bytes() == C.sizeof(lb.lb_params)


def test_workspace_bytes_scales_with_storage():
    wl, *_ = W.taylor_green_blobs()
    b64 = lb.lb_workspace_bytes(lb.params_from_workload(wl, "f64"))
    b32 = lb.lb_workspace_bytes(lb.params_from_workload(wl, "f32"))
    b16 = lb.lb_workspace_bytes(lb.params_from_workload(wl, "f16", fp16_scale=100.0))
    assert b64 > b32 > b16 > 19 * 64 * 64 * 2


@pytest.mark.parametrize("mutate, status", [
    (lambda p: setattr(p, "tau_f", 0.5), lb.LB_EINVAL),
    (lambda p: setattr(p, "m", 5), lb.LB_EINVAL),
    (lambda p: setattr(p, "nx", 1), lb.LB_EINVAL),
    (lambda p: p.D.__setitem__(0, -0.01), lb.LB_EINVAL),        # eigenvalue with negative real part
    (lambda p: p.fluid_bc.__setitem__(0, 1), lb.LB_EINVAL),     # half a periodic pair
    (lambda p: setattr(p, "storage", 7), lb.LB_EINVAL),
    (lambda p: setattr(p, "fused_steps", 3), lb.LB_EINVAL),
])
def test_validation_rejects(mutate, status):
    wl, *_ = W.taylor_green_blobs()
    p = lb.params_from_workload(wl)
    mutate(p)
    with pytest.raises(lb.LBError) as ei:
        lb.lb_workspace_bytes(p)
    assert ei.value.status == status
    assert lb.lib().lb_last_error()


def test_complex_eigenvalues_with_positive_real_part_accepted():
    wl = W._base(8, 8, 2, 0.8, [[0.05, 0.04], [-0.04, 0.05]])  # eig 0.05 +- 0.04i
    assert lb.lb_workspace_bytes(lb.params_from_workload(wl)) > 0


def test_init_rejects_before_touching_the_device():
    wl, phi0, u0, p0 = W.taylor_green_blobs()
    p = lb.params_from_workload(wl)
    n = lb.lb_workspace_bytes(p)
    h = C.c_void_p()
    L = lb.lib()
    # NULL workspace
    st = L.lb_init(C.byref(p), None, n, None, phi0.ctypes.data, u0.ctypes.data, None, C.byref(h))
    assert st == lb.LB_EINVAL and not h.value
    # misaligned workspace
    st = L.lb_init(C.byref(p), C.c_void_p(0x1008), n, None, phi0.ctypes.data, u0.ctypes.data, None, C.byref(h))
    assert st == lb.LB_EINVAL
    # too small
    st = L.lb_init(C.byref(p), C.c_void_p(0x10000), n - 1, None, phi0.ctypes.data, u0.ctypes.data, None, C.byref(h))
    assert st == lb.LB_ENOMEM
    # non-finite initial field (checked on the host, before any copy)
    bad = np.ascontiguousarray(phi0.copy())
    bad[1, 3, 4] = np.nan
    st = L.lb_init(C.byref(p), C.c_void_p(0x10000), n, None, bad.ctypes.data, u0.ctypes.data, None, C.byref(h))
    assert st == lb.LB_ENONFINITE and not h.value


def test_free_null_is_ok():
    assert lb.lib().lb_free(None) == lb.LB_OK


@pytest.mark.parametrize("mutate", [
    lambda p: setattr(p, "storage", lb.STORAGE["f16"]) or setattr(p, "fp16_scale", 1.0) or setattr(p, "fp16_scale_h", 1.0),
    lambda p: setattr(p, "collision", 1),
    lambda p: setattr(p, "fused_steps", 2),
    lambda p: p.F0.__setitem__(1, 1e-5),
    lambda p: p.Fphi[0].__setitem__(1, 1e-5),
])
def test_no_fluid_model_validation(mutate):
    wl, *_ = W.cde_case(16, 12)
    p = lb.params_from_workload(wl)
    assert lb.lb_workspace_bytes(p) > 0
    mutate(p)
    with pytest.raises(lb.LBError) as ei:
        lb.lb_workspace_bytes(p)
    assert ei.value.status == lb.LB_EINVAL


def test_no_fluid_model_needs_no_fluid_planes():
    wl, *_ = W.cde_case(64, 64)
    b_cde = lb.lb_workspace_bytes(lb.params_from_workload(wl))
    wl["model"] = "linear"
    b_lin = lb.lb_workspace_bytes(lb.params_from_workload(wl))
    assert b_cde < b_lin


def _set_lam(p, m, lam):
    for a in range(m):
        for b in range(m):
            p.lam[a * m + b] = lam[a][b]


def test_lambda_and_varphi_accepted():
    wl, *_ = W.taylor_green_blobs()
    p = lb.params_from_workload(wl)
    _set_lam(p, 2, [[0.6, 0.3], [-0.1, 1.2]])
    p.varphi = 1.0
    assert lb.lb_workspace_bytes(p) > 0
    wl, *_ = W.cde_case(16, 12)
    p = lb.params_from_workload(wl)
    _set_lam(p, wl["m"], np.eye(wl["m"]) * 0.9)
    assert lb.lb_workspace_bytes(p) > 0


@pytest.mark.parametrize("case", ["singular", "rest_weight", "negative", "chemotaxis", "mrt_varphi",
                                  "cde_varphi", "nonfinite"])
def test_lambda_and_varphi_validation(case):
    if case == "chemotaxis":
        wl, *_ = W.random_case(16, 12, m=2, seed=1, model="chemotaxis")
    elif case == "cde_varphi":
        wl, *_ = W.cde_case(16, 12)
    else:
        wl, *_ = W.taylor_green_blobs()
    p = lb.params_from_workload(wl)
    m = wl["m"]
    lam = {"singular": [[1.0, 1.0], [1.0, 1.0]], "rest_weight": [[1.6, 0.0], [0.0, 1.0]],
           "negative": [[1.0, 0.0], [0.0, -0.5]], "chemotaxis": [[0.9, 0.0], [0.0, 1.0]]}.get(case)
    if lam is not None:
        _set_lam(p, m, lam)
    if case == "mrt_varphi":
        p.collision = 1
        p.varphi = 1.0
    if case == "cde_varphi":
        p.varphi = 1.0
    if case == "nonfinite":
        p.varphi = float("nan")
    with pytest.raises(lb.LBError) as ei:
        lb.lb_workspace_bytes(p)
    assert ei.value.status == lb.LB_EINVAL


# ---- 3-D library (include/lb3.h) ------------------------------------------
def test_lb3_params_record_matches():
    from paper_2101_03055_amd import lb3
    assert lb3.lib().lb3_params_bytes() == C.sizeof(lb3.lb3_params)


@pytest.mark.parametrize("case", ["tau", "m", "grid", "half_pair", "freeslip", "f16", "eig", "nonfinite",
                                  "scalar_periodic_mismatch"])
def test_lb3_validation_rejects(case):
    from paper_2101_03055_amd import lb3
    wl, *_ = W.random_case3(12, 10, 8, m=2, seed=3)
    p = lb3.params_from_workload(wl)
    assert lb3.lb3_workspace_bytes(p) > 0
    if case == "tau":
        p.tau_f = 0.5
    elif case == "m":
        p.m = 5
    elif case == "grid":
        p.nz = 1
    elif case == "half_pair":
        p.fluid_bc[4] = 1
    elif case == "freeslip":
        p.fluid_bc[4] = p.fluid_bc[5] = 2
    elif case == "f16":
        p.storage = 2
    elif case == "eig":
        p.D[0] = -0.2
    elif case == "nonfinite":
        p.F0[2] = float("inf")
    elif case == "scalar_periodic_mismatch":
        p.fluid_bc[4] = p.fluid_bc[5] = 1
    with pytest.raises(lb.LBError) as ei:
        lb3.lb3_workspace_bytes(p)
    assert ei.value.status == lb.LB_EINVAL
    assert lb3.lib().lb3_last_error()


def test_lb3_init_rejects_before_touching_the_device():
    from paper_2101_03055_amd import lb3
    wl, phi0, u0, p0 = W.random_case3(12, 10, 8, m=2, seed=3)
    p = lb3.params_from_workload(wl)
    n = lb3.lb3_workspace_bytes(p)
    h = C.c_void_p()
    L = lb3.lib()
    phi0 = np.ascontiguousarray(phi0)
    u0 = np.ascontiguousarray(u0)
    assert L.lb3_init(C.byref(p), None, n, None, phi0.ctypes.data, u0.ctypes.data, None, C.byref(h)) == lb.LB_EINVAL
    assert L.lb3_init(C.byref(p), C.c_void_p(0x1008), n, None, phi0.ctypes.data, u0.ctypes.data, None,
                      C.byref(h)) == lb.LB_EINVAL
    assert L.lb3_init(C.byref(p), C.c_void_p(0x10000), n - 1, None, phi0.ctypes.data, u0.ctypes.data, None,
                      C.byref(h)) == lb.LB_ENOMEM
    bad = phi0.copy()
    bad[0, 1, 2, 3] = np.nan
    assert L.lb3_init(C.byref(p), C.c_void_p(0x10000), n, None, bad.ctypes.data, u0.ctypes.data, None,
                      C.byref(h)) == lb.LB_ENONFINITE
    assert not h.value
    assert L.lb3_free(None) == lb.LB_OK


def test_gamma_validation():
    """gamma of D-bar: finite, not with two steps per launch, the no-fluid
    model or a batch; a species without a source makes gamma inert (no second
    source buffer)."""
    wl, *_ = W.random_case(16, 12, m=2, seed=1, source=True)
    base = lb.params_from_workload(dict(wl, gamma_s=[0.0, 0.0]))
    p = lb.params_from_workload(dict(wl, gamma_s=[1.0, -0.5]))
    assert lb.lb_workspace_bytes(p) > lb.lb_workspace_bytes(base)      # the second source buffer
    nan = lb.params_from_workload(dict(wl, gamma_s=[float("nan"), 0.0]))
    fused = lb.params_from_workload(dict(wl, gamma_s=[1.0, 0.0]), fused_steps=2)
    for bad in (nan, fused):
        with pytest.raises(lb.LBError) as ei:
            lb.lb_workspace_bytes(bad)
        assert ei.value.status == lb.LB_EINVAL
    with pytest.raises(lb.LBError) as ei:
        lb.lbb_workspace_bytes([p, p])
    assert ei.value.status == lb.LB_EINVAL
    nosrc, *_ = W.random_case(16, 12, m=2, seed=1, source=False)
    assert lb.lb_workspace_bytes(lb.params_from_workload(dict(nosrc, gamma_s=[1.0, 1.0]))) == \
        lb.lb_workspace_bytes(lb.params_from_workload(nosrc))
