"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Two child processes, each with its sanitizer runtime preloaded:
  * the oracle built by gcc with -fsanitize=address,undefined, run through
    every model, boundary kind, collision and planted mistake;
  * the HIP library with its host code instrumented (device code untouched),
    run through every host path that needs no GPU: parameter validation
    (eigenvalues, inverses, layouts) for valid and invalid records, workspace
    sizes of single domains, batches and the surrogate.
A sanitizer report makes the child exit non-zero.
"""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
pytestmark = pytest.mark.slow

ENV_SAN = {"ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:verify_asan_link_order=0",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def run_child(code, extra_env):
    env = dict(os.environ, **ENV_SAN, **extra_env, PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, "-c", textwrap.dedent(code)], env=env, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 0 and "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, \
        r.stdout[-2000:] + r.stderr[-4000:]
    return r.stdout


def test_oracle_under_asan_ubsan(tmp_path):
    lib = str(tmp_path / "liblboracle_san.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                           "-fno-omit-frame-pointer", os.path.join(ROOT, "oracle", "lb_oracle.c"), "-o", lib, "-lm"])
    assert "__asan_report" in subprocess.check_output(["nm", "-D", lib], text=True)  # instrumented
    asan = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    ubsan = subprocess.check_output(["gcc", "-print-file-name=libubsan.so"], text=True).strip()
    out = run_child("""
        import numpy as np
        from oracle import oracle as O
        from paper_2101_03055_amd import workloads as W
        cases = [W.random_case(13, 9, seed=1, fluid_bc=["noslip", "freeslip", "noslip", "freeslip"],
                               scalar_bc=[["dirichlet"] * 2, ["noflux"] * 2, ["dirichlet"] * 2, ["noflux"] * 2],
                               source=True),
                 W.random_case(12, 10, seed=2, model="chemotaxis", collision="mrt",
                               fluid_bc=["periodic", "periodic", "noslip", "freeslip"],
                               scalar_bc=[["periodic"] * 2, ["periodic"] * 2, ["noflux"] * 2, ["noflux", "dirichlet"]]),
                 W.random_case(11, 7, m=4, seed=3),
                 W.cde_case(10, 8, m=3, seed=4, walls=True, source=True)]
        for wl, phi0, u0, p0 in cases:
            for mut in (0, 1, 7, 9):
                o = O.Oracle(wl, phi0, u0, p0, mutation=mut)
                o.step(3)
                o.moments()
        print("oracle ok")
    """, {"LD_PRELOAD": f"{asan}:{ubsan}", "LB_ORACLE_LIBRARY": lib})
    assert "oracle ok" in out


def test_library_host_code_under_asan_ubsan(tmp_path):
    from paper_2101_03055_amd import build as B

    libs = B.build(sanitize=True, out_dir=str(tmp_path))
    assert "__asan_report" in subprocess.check_output(["nm", "-D", libs[0]], text=True)  # host code instrumented
    clang = subprocess.check_output(["/opt/rocm/llvm/bin/clang", "-print-resource-dir"], text=True).strip()
    asan = os.path.join(clang, "lib", "linux", "libclang_rt.asan-x86_64.so")
    assert os.path.exists(asan)
    out = run_child("""
        import copy
        import numpy as np
        from paper_2101_03055_amd import lb, sg, workloads as W
        good = [W.taylor_green_blobs()[0], W.chemotaxis_plume()[0], W.ddc_cavity(64)[0], W.cde_case(32, 24)[0],
                W.random_case(9, 7, m=4, seed=5, collision="mrt")[0]]
        n_ok = n_bad = 0
        for wl in good:
            for storage in ("f64", "f32", "f16"):
                try:
                    p = lb.params_from_workload(wl, storage, fp16_scale=10.0)
                    lb.lb_workspace_bytes(p)
                    n_ok += 1
                except lb.LBError:
                    n_bad += 1  # e.g. F16 for the no-fluid model
            p = lb.params_from_workload(wl)
            for field, value in (("tau_f", 0.5), ("m", 0), ("m", 9), ("nx", 1), ("storage", 5), ("fused_steps", 4),
                                 ("collision", 3), ("model", 7), ("r_kind", 4)):
                q = copy.copy(p)
                setattr(q, field, value)
                try:
                    lb.lb_workspace_bytes(q)
                except lb.LBError:
                    n_bad += 1
                    assert lb.lib().lb_last_error()
        params = [lb.params_from_workload(W.ddc_case(pd)[0], "f32") for pd in W.sweep_params(12, seed=3)]
        arr = (lb.lb_params * len(params))(*params)
        import ctypes as C
        nb = C.c_size_t()
        assert lb.lib().lbb_workspace_bytes(arr, len(params), C.byref(nb)) == 0 and nb.value > 0
        assert sg.param_count()[0] > 0
        for l in range(sg.SG_LAYERS):
            sg.layer_info(l)
        cfg = sg.sg_config(4, 64, 128, 0, 1e-3, 0.9, 0.999, 1e-8)
        assert sg.lib().sg_workspace_bytes(C.byref(cfg), C.byref(nb)) == 0 and nb.value > 0
        print("host ok", n_ok, n_bad)
    """, {"LD_PRELOAD": asan, "LBCDF_LIBRARY": libs[0]})
    assert "host ok" in out
