"""Python binding of the C ABI in include/lb.h (argument marshalling only).

Functions carry the C names (``lb_init``, ``lb_step``, ...).  Device memory
and the stream come from PyTorch: the workspace is a ``torch.uint8`` CUDA
tensor and the stream is ``torch.cuda.current_stream().cuda_stream``.  Every
step of the method runs in the HIP kernels of ``liblbcdf.so``; this module
raises if that library is missing or fails to load.

``Solver`` bundles the handle with its workspace for convenience.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# LBCDF_LIBRARY selects another build of the same library (the host-sanitized
# copy used by the sanitizer test); by default the in-tree build is loaded
LIBPATH = os.environ.get("LBCDF_LIBRARY") or os.path.join(HERE, "liblbcdf.so")
MAXM = 4

LB_OK, LB_EINVAL, LB_ENOMEM, LB_EDEVICE, LB_ENONFINITE, LB_ESTATE = 0, -1, -2, -3, -4, -5
MODEL = {"linear": 0, "chemotaxis": 1, "cde": 2}
STORAGE = {"f64": 0, "f32": 1, "f16": 2}
COLLISION = {"bgk": 0, "mrt": 1}
RKIND = {"step": 0, "smooth": 1}
FLUID_BC = {"periodic": 0, "noslip": 1, "freeslip": 2}
SCALAR_BC = {"periodic": 0, "noflux": 1, "dirichlet": 2}


class LBError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"lb status {status}: {msg}")
        self.status = status


class lb_params(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("m", C.c_int32), ("model", C.c_int32),
        ("storage", C.c_int32), ("collision", C.c_int32), ("r_kind", C.c_int32),
        ("fluid_bc", C.c_int32 * 4),
        ("scalar_bc", (C.c_int32 * MAXM) * 4),
        ("fused_steps", C.c_int32),
        ("tau_f", C.c_double), ("rho0", C.c_double),
        ("mrt_s", C.c_double * 9),
        ("D", C.c_double * (MAXM * MAXM)),
        ("K", C.c_double * (MAXM * MAXM)),
        ("F0", C.c_double * 2),
        ("Fphi", (C.c_double * 2) * MAXM),
        ("chi", C.c_double), ("beta", C.c_double), ("cstar", C.c_double), ("eps", C.c_double),
        ("wall", (C.c_double * MAXM) * 4),
        ("phi_ref", C.c_double * MAXM),
        ("fp16_scale", C.c_double),
        ("fp16_scale_h", C.c_double),
        ("lam", C.c_double * (MAXM * MAXM)),
        ("varphi", C.c_double),
        ("gamma_s", C.c_double * MAXM),
    ]


_lib = None


def lib():
    """The loaded HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            raise RuntimeError(f"{LIBPATH} is missing: run `python -m paper_2101_03055_amd.build` "
                               "(there is no CPU fallback)")
        L = C.CDLL(LIBPATH)
        vp, sz, i64, st = C.c_void_p, C.c_size_t, C.c_int64, C.c_int
        pp = C.POINTER(lb_params)
        sig = {
            "lb_workspace_bytes": [pp, C.POINTER(sz)],
            "lb_init": [pp, vp, sz, vp, vp, vp, vp, C.POINTER(vp)],
            "lb_step": [vp, i64],
            "lb_moments": [vp, vp, vp, vp],
            "lb_moments_device": [vp, vp, vp, vp],
            "lb_residual": [vp, vp],
            "lb_residual_noalloc": [vp, vp],
            "lb_mass": [vp, vp],
            "lb_populations": [vp, vp, vp],
            "lb_time": [vp, C.POINTER(i64)],
            "lb_state_bytes": [vp, C.POINTER(sz)],
            "lb_save": [vp, vp, sz],
            "lb_load": [vp, vp, sz],
            "lb_set_tile": [vp, C.c_int32, C.c_int32],
            "lb_copy_state": [vp, vp],
            "lb_fluid_reference": [vp, C.c_int32],
            "lb_wall_flux": [vp, C.c_int32, vp],
            "lb_solve_steady": [vp, C.c_double, i64, i64, C.POINTER(i64), vp],
            "lb_free": [vp],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = st
        pvp = C.POINTER(C.c_void_p)
        bsig = {
            "lbb_workspace_bytes": [pp, C.c_int32, C.POINTER(sz)],
            "lbb_init": [pp, C.c_int32, vp, sz, vp, pvp, pvp, pvp, C.POINTER(vp)],
            "lbb_step": [vp, i64],
            "lbb_run": [vp, C.c_double, i64, i64, vp, vp, vp],
            "lbb_moments": [vp, C.c_int32, vp, vp, vp],
            "lbb_time": [vp, C.c_int32, C.POINTER(i64), C.POINTER(C.c_int32)],
            "lbb_copy_cavity": [vp, C.c_int32, vp, C.c_int32],
            "lbb_set_tile": [vp, C.c_int32, C.c_int32],
            "lbb_autotune": [vp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_double)],
            "lbb_cavity_tile": [vp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)],
            "lbb_set_cavity_tile": [vp, C.c_int32, C.c_int32, C.c_int32],
            "lbb_free": [vp],
        }
        for name, args in bsig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = st
        L.lb_last_error.restype = C.c_char_p
        L.lb_params_bytes.restype = sz
        if L.lb_params_bytes() != C.sizeof(lb_params):
            raise RuntimeError("lb_params mirror does not match the library")
        _lib = L
    return _lib


def _check(status):
    if status != LB_OK:
        raise LBError(status, lib().lb_last_error().decode())


def params_from_workload(wl: dict, storage: str = "f64", phi_ref=None, fp16_scale: float = 1.0,
                         fp16_scale_h: float | None = None, fused_steps: int = 0) -> lb_params:
    """Fill the C record from a workload dict (see ``workloads``)."""
    p = lb_params()
    m = wl["m"]
    p.nx, p.ny, p.m = wl["nx"], wl["ny"], m
    p.model = MODEL[wl.get("model", "linear")]
    p.storage = STORAGE[storage]
    p.collision = COLLISION[wl.get("collision", "bgk")]
    p.r_kind = RKIND[wl.get("r_kind", "step")]
    fb = wl.get("fluid_bc", ["periodic"] * 4)
    sb = wl.get("scalar_bc", [["periodic"] * m] * 4)
    for s in range(4):
        p.fluid_bc[s] = FLUID_BC[fb[s]]
        for a in range(m):
            p.scalar_bc[s][a] = SCALAR_BC[sb[s][a]]
    p.tau_f = wl["tau_f"]
    p.rho0 = wl.get("rho0", 1.0)
    for k, v in enumerate(wl.get("mrt_s", [1.0] * 9)):
        p.mrt_s[k] = v
    D = np.asarray(wl["D"], dtype=np.float64).reshape(m, m)
    K = np.asarray(wl.get("K", np.zeros((m, m))), dtype=np.float64).reshape(m, m)
    for a in range(m):
        for b in range(m):
            p.D[a * m + b] = D[a, b]
            p.K[a * m + b] = K[a, b]
    p.F0[0], p.F0[1] = wl.get("F0", [0.0, 0.0])
    Fphi = np.asarray(wl.get("Fphi", np.zeros((m, 2))), dtype=np.float64).reshape(m, 2)
    for a in range(m):
        p.Fphi[a][0], p.Fphi[a][1] = Fphi[a]
    p.chi, p.beta = wl.get("chi", 0.0), wl.get("beta", 0.0)
    p.cstar, p.eps = wl.get("cstar", 0.3), wl.get("eps", 0.0)
    wall = np.asarray(wl.get("wall", np.zeros((4, m))), dtype=np.float64).reshape(4, m)
    for s in range(4):
        for a in range(m):
            p.wall[s][a] = wall[s, a]
    if phi_ref is not None:
        for a in range(m):
            p.phi_ref[a] = float(phi_ref[a])
    p.fp16_scale = fp16_scale
    p.fp16_scale_h = fp16_scale if fp16_scale_h is None else fp16_scale_h
    p.fused_steps = int(fused_steps)
    if "lam" in wl:
        lam = np.asarray(wl["lam"], dtype=np.float64).reshape(m, m)
        for a in range(m):
            for b in range(m):
                p.lam[a * m + b] = lam[a, b]
    p.varphi = float(wl.get("varphi", 0.0))
    for a, g in enumerate(wl.get("gamma_s", [0.0] * m)):
        p.gamma_s[a] = float(g)
    return p


# ---- thin wrappers with the C names ------------------------------------------
def lb_workspace_bytes(p: lb_params) -> int:
    n = C.c_size_t()
    _check(lib().lb_workspace_bytes(C.byref(p), C.byref(n)))
    return n.value


def _host(a, shape):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.size != int(np.prod(shape)):
        raise ValueError(f"array of {a.size} values, {shape} expected")
    return a


def lb_init(p: lb_params, workspace_ptr: int, workspace_bytes: int, stream: int, phi0, u0, p0=None):
    m, ny, nx = p.m, p.ny, p.nx
    phi0 = _host(phi0, (m, ny, nx))
    u0 = _host(u0, (2, ny, nx))
    p0a = None if p0 is None else _host(p0, (ny, nx))
    h = C.c_void_p()
    _check(lib().lb_init(C.byref(p), C.c_void_p(workspace_ptr), workspace_bytes, C.c_void_p(stream),
                         phi0.ctypes.data, u0.ctypes.data, None if p0a is None else p0a.ctypes.data,
                         C.byref(h)))
    return h


def lb_step(h, n: int):
    _check(lib().lb_step(h, int(n)))


def lb_moments(h, m: int, ny: int, nx: int):
    phi = np.empty((m, ny, nx))
    u = np.empty((2, ny, nx))
    pr = np.empty((ny, nx))
    _check(lib().lb_moments(h, phi.ctypes.data, u.ctypes.data, pr.ctypes.data))
    return phi, u, pr


def lb_moments_device(h, d_phi: int, d_u: int, d_p: int):
    _check(lib().lb_moments_device(h, C.c_void_p(d_phi or None), C.c_void_p(d_u or None), C.c_void_p(d_p or None)))


def lb_residual(h, m: int):
    """Returns (res[m + 2], status); status LB_ENONFINITE is reported, not raised."""
    res = np.empty(m + 2)
    st = lib().lb_residual(h, res.ctypes.data)
    if st not in (LB_OK, LB_ENONFINITE):
        _check(st)
    return res, st


def lb_residual_noalloc(h, m: int):
    """lb_residual through the entry point that allocates nothing (library-held
    scratch array); returns (res[m + 2], status) like lb_residual."""
    res = np.empty(m + 2)
    st = lib().lb_residual_noalloc(h, res.ctypes.data)
    if st not in (LB_OK, LB_ENONFINITE):
        _check(st)
    return res, st


def lb_mass(h, m: int):
    out = np.empty(m + 1)
    st = lib().lb_mass(h, out.ctypes.data)
    if st not in (LB_OK, LB_ENONFINITE):
        _check(st)
    return out, st


def lb_populations(h, m: int, ny: int, nx: int):
    f = np.empty((m, 5, ny, nx))
    hp = np.empty((9, ny, nx))
    _check(lib().lb_populations(h, f.ctypes.data, hp.ctypes.data))
    return f, hp


def lb_time(h) -> int:
    t = C.c_int64()
    _check(lib().lb_time(h, C.byref(t)))
    return t.value


def lb_save(h) -> bytes:
    n = C.c_size_t()
    _check(lib().lb_state_bytes(h, C.byref(n)))
    buf = C.create_string_buffer(n.value)
    _check(lib().lb_save(h, buf, n.value))
    return buf.raw


def lb_load(h, blob: bytes):
    buf = C.create_string_buffer(blob, len(blob))
    _check(lib().lb_load(h, buf, len(blob)))


def lb_solve_steady(h, m: int, tol: float, check_every: int, max_steps: int):
    """Returns (steps, res[m + 2], status) with status LB_OK (converged),
    LB_ESTATE (step cap reached) or LB_ENONFINITE (diverged)."""
    steps = C.c_int64()
    res = np.full(m + 2, np.inf)
    st = lib().lb_solve_steady(h, float(tol), int(check_every), int(max_steps), C.byref(steps), res.ctypes.data)
    if st not in (LB_OK, LB_ESTATE, LB_ENONFINITE):
        _check(st)
    return steps.value, res, st


def lb_wall_flux(h, side: int, m: int):
    out = np.empty(m)
    _check(lib().lb_wall_flux(h, int(side), out.ctypes.data))
    return out


def lb_copy_state(dst, src):
    _check(lib().lb_copy_state(dst, src))


def lb_fluid_reference(h, mode: int = 1):
    _check(lib().lb_fluid_reference(h, int(mode)))


def lb_set_tile(h, tile_x: int, tile_y: int):
    _check(lib().lb_set_tile(h, int(tile_x), int(tile_y)))


def lb_free(h):
    lib().lb_free(h)


class Solver:
    """A handle plus the torch workspace that backs it (freed together)."""

    def __init__(self, wl: dict, phi0, u0, p0=None, storage: str = "f64", phi_ref=None,
                 fp16_scale: float = 1.0, fp16_scale_h: float | None = None, device: str = "cuda:0",
                 stream=None, fused_steps: int = 0):
        import torch

        lib()
        self.wl = wl
        self.m, self.ny, self.nx = wl["m"], wl["ny"], wl["nx"]
        self.params = params_from_workload(wl, storage, phi_ref, fp16_scale, fp16_scale_h, fused_steps)
        nbytes = lb_workspace_bytes(self.params)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.workspace.device)
        self.handle = lb_init(self.params, self.workspace.data_ptr(), nbytes, self.stream.cuda_stream,
                              phi0, u0, p0)

    def step(self, n: int):
        lb_step(self.handle, n)

    def moments(self):
        return lb_moments(self.handle, self.m, self.ny, self.nx)

    def residual(self):
        return lb_residual(self.handle, self.m)

    def mass(self):
        return lb_mass(self.handle, self.m)

    def fluid_reference(self, mode: int = 1):
        """Store the fluid relative to the current row-mean pressure (mode 1) or
        to no reference (mode 0); see lb_fluid_reference."""
        lb_fluid_reference(self.handle, mode)

    def solve_steady(self, tol=1e-8, check_every=1000, max_steps=5_000_000):
        return lb_solve_steady(self.handle, self.m, tol, check_every, max_steps)

    def populations(self):
        return lb_populations(self.handle, self.m, self.ny, self.nx)

    @property
    def t(self) -> int:
        return lb_time(self.handle)

    def close(self):
        if getattr(self, "handle", None) is not None:
            lb_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- batched sweep -------------------------------------------------------------
LBB_RUNNING, LBB_CONVERGED, LBB_DIVERGED = 0, 1, 2


def _params_array(plist):
    arr = (lb_params * len(plist))()
    for k, q in enumerate(plist):
        arr[k] = q
    return arr


def lbb_workspace_bytes(plist) -> int:
    arr = _params_array(plist)
    n = C.c_size_t()
    _check(lib().lbb_workspace_bytes(arr, len(plist), C.byref(n)))
    return n.value


def lbb_init(plist, workspace_ptr: int, workspace_bytes: int, stream: int, phi0s, u0s, p0s=None):
    arr = _params_array(plist)
    cnt = len(plist)
    keep = []

    def ptrs(arrays, shapes):
        out = (C.c_void_p * cnt)()
        for k in range(cnt):
            if arrays is None or arrays[k] is None:
                out[k] = None
                continue
            a = _host(arrays[k], shapes[k])
            keep.append(a)
            out[k] = a.ctypes.data
        return out

    sh_phi = [(q.m, q.ny, q.nx) for q in plist]
    sh_u = [(2, q.ny, q.nx) for q in plist]
    sh_p = [(q.ny, q.nx) for q in plist]
    h = C.c_void_p()
    _check(lib().lbb_init(arr, cnt, C.c_void_p(workspace_ptr), workspace_bytes, C.c_void_p(stream),
                          ptrs(phi0s, sh_phi), ptrs(u0s, sh_u), None if p0s is None else ptrs(p0s, sh_p),
                          C.byref(h)))
    return h


def lbb_step(b, n: int):
    _check(lib().lbb_step(b, int(n)))


def lbb_run(b, count: int, m: int, tol: float, check_every: int, max_steps: int):
    steps = np.zeros(count, dtype=np.int64)
    status = np.zeros(count, dtype=np.int32)
    res = np.zeros((count, m + 2))
    _check(lib().lbb_run(b, float(tol), int(check_every), int(max_steps), steps.ctypes.data, status.ctypes.data,
                         res.ctypes.data))
    return steps, status, res


def lbb_moments(b, i: int, m: int, ny: int, nx: int):
    phi = np.empty((m, ny, nx))
    u = np.empty((2, ny, nx))
    pr = np.empty((ny, nx))
    _check(lib().lbb_moments(b, int(i), phi.ctypes.data, u.ctypes.data, pr.ctypes.data))
    return phi, u, pr


def lbb_time(b, i: int):
    s = C.c_int64()
    st = C.c_int32()
    _check(lib().lbb_time(b, int(i), C.byref(s), C.byref(st)))
    return s.value, st.value


def lbb_copy_cavity(dst, i: int, src, j: int):
    _check(lib().lbb_copy_cavity(dst, int(i), src, int(j)))


def lbb_set_tile(b, tile_x: int, tile_y: int):
    _check(lib().lbb_set_tile(b, int(tile_x), int(tile_y)))


def lbb_autotune(b, trial_steps: int = 20):
    tx, ty, us = C.c_int32(), C.c_int32(), C.c_double()
    _check(lib().lbb_autotune(b, int(trial_steps), C.byref(tx), C.byref(ty), C.byref(us)))
    return tx.value, ty.value, us.value


def lbb_set_cavity_tile(b, i: int, tile_x: int, tile_y: int):
    _check(lib().lbb_set_cavity_tile(b, int(i), int(tile_x), int(tile_y)))


def lbb_cavity_tile(b, i: int):
    tx, ty = C.c_int32(), C.c_int32()
    _check(lib().lbb_cavity_tile(b, int(i), C.byref(tx), C.byref(ty)))
    return tx.value, ty.value


def lbb_free(b):
    lib().lbb_free(b)


class Batch:
    """A batch handle plus its torch workspace."""

    def __init__(self, cases, storage: str = "f64", phi_ref=None, fp16_scale: float = 1.0,
                 fp16_scale_h=None, device: str = "cuda:0", stream=None):
        """cases: list of (workload dict, phi0, u0, p0)."""
        import torch

        lib()
        self.wls = [c[0] for c in cases]
        self.count = len(cases)
        self.m = self.wls[0]["m"]
        self.params = [params_from_workload(wl, storage, phi_ref, fp16_scale, fp16_scale_h) for wl in self.wls]
        nbytes = lbb_workspace_bytes(self.params)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.workspace.device)
        self.handle = lbb_init(self.params, self.workspace.data_ptr(), nbytes, self.stream.cuda_stream,
                               [c[1] for c in cases], [c[2] for c in cases], [c[3] for c in cases])

    def step(self, n: int):
        lbb_step(self.handle, n)

    def run(self, tol=1e-8, check_every=1000, max_steps=5_000_000):
        return lbb_run(self.handle, self.count, self.m, tol, check_every, max_steps)

    def moments(self, i: int):
        wl = self.wls[i]
        return lbb_moments(self.handle, i, self.m, wl["ny"], wl["nx"])

    def time(self, i: int):
        return lbb_time(self.handle, i)

    def autotune(self, trial_steps: int = 20):
        return lbb_autotune(self.handle, trial_steps)

    def cavity_tile(self, i: int):
        """Tile shape (tile_x, tile_y) the batched step uses for cavity i."""
        return lbb_cavity_tile(self.handle, i)

    def close(self):
        if getattr(self, "handle", None) is not None:
            lbb_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
