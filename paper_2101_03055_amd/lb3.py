"""Thin ctypes binding of include/lb3.h (the 3-D model: D3Q7 scalars, D3Q19
fluid).  Argument marshalling only: every step runs in the HIP library; there
is no CPU fallback (a missing library raises)."""
from __future__ import annotations

import ctypes as C

import numpy as np

from .lb import FLUID_BC, LBError, LB_OK, SCALAR_BC, STORAGE, lib as _lib2

MAXM = 4


class lb3_params(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("m", C.c_int32), ("storage", C.c_int32),
        ("fluid_bc", C.c_int32 * 6),
        ("scalar_bc", (C.c_int32 * MAXM) * 6),
        ("pad_", C.c_int32),
        ("tau_f", C.c_double), ("rho0", C.c_double),
        ("D", C.c_double * (MAXM * MAXM)),
        ("K", C.c_double * (MAXM * MAXM)),
        ("F0", C.c_double * 3),
        ("Fphi", (C.c_double * 3) * MAXM),
        ("wall", (C.c_double * MAXM) * 6),
        ("phi_ref", C.c_double * MAXM),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = _lib2()
        vp, sz, i64, st = C.c_void_p, C.c_size_t, C.c_int64, C.c_int
        pp = C.POINTER(lb3_params)
        sig = {
            "lb3_workspace_bytes": [pp, C.POINTER(sz)],
            "lb3_init": [pp, vp, sz, vp, vp, vp, vp, C.POINTER(vp)],
            "lb3_step": [vp, i64],
            "lb3_moments": [vp, vp, vp, vp],
            "lb3_populations": [vp, vp, vp],
            "lb3_mass": [vp, vp],
            "lb3_time": [vp, C.POINTER(i64)],
            "lb3_set_tile": [vp, C.c_int32, C.c_int32],
            "lb3_free": [vp],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = st
        L.lb3_last_error.restype = C.c_char_p
        L.lb3_params_bytes.restype = sz
        if L.lb3_params_bytes() != C.sizeof(lb3_params):
            raise RuntimeError("lb3_params mirror does not match the library")
        _lib = L
    return _lib


def _check(status):
    if status != LB_OK:
        raise LBError(status, lib().lb3_last_error().decode())


def params_from_workload(wl: dict, storage: str = "f64", phi_ref=None) -> lb3_params:
    p = lb3_params()
    m = wl["m"]
    p.nx, p.ny, p.nz, p.m = wl["nx"], wl["ny"], wl["nz"], m
    p.storage = STORAGE[storage]
    fb = wl.get("fluid_bc", ["periodic"] * 6)
    sb = wl.get("scalar_bc", [["periodic"] * m] * 6)
    for s in range(6):
        p.fluid_bc[s] = FLUID_BC[fb[s]]
        for a in range(m):
            p.scalar_bc[s][a] = SCALAR_BC[sb[s][a]]
    p.tau_f = wl["tau_f"]
    p.rho0 = wl.get("rho0", 1.0)
    D = np.asarray(wl["D"], dtype=np.float64).reshape(m, m)
    K = np.asarray(wl.get("K", np.zeros((m, m))), dtype=np.float64).reshape(m, m)
    for a in range(m):
        for b in range(m):
            p.D[a * m + b] = D[a, b]
            p.K[a * m + b] = K[a, b]
    for d, v in enumerate(wl.get("F0", [0.0, 0.0, 0.0])):
        p.F0[d] = v
    Fphi = np.asarray(wl.get("Fphi", np.zeros((m, 3))), dtype=np.float64).reshape(m, 3)
    wall = np.asarray(wl.get("wall", np.zeros((6, m))), dtype=np.float64).reshape(6, m)
    for a in range(m):
        for d in range(3):
            p.Fphi[a][d] = Fphi[a, d]
        for s in range(6):
            p.wall[s][a] = wall[s, a]
        if phi_ref is not None:
            p.phi_ref[a] = float(phi_ref[a])
    return p


def lb3_workspace_bytes(p: lb3_params) -> int:
    n = C.c_size_t()
    _check(lib().lb3_workspace_bytes(C.byref(p), C.byref(n)))
    return n.value


def _f64(a, shape):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.size != int(np.prod(shape)):
        raise ValueError(f"expected {shape}, got {a.shape}")
    return a


class Solver3:
    """A 3-D handle plus the torch workspace that backs it (freed together)."""

    def __init__(self, wl: dict, phi0, u0, p0=None, storage: str = "f64", phi_ref=None, device: str = "cuda:0",
                 stream=None):
        import torch

        self.wl = wl
        self.m, self.nz, self.ny, self.nx = wl["m"], wl["nz"], wl["ny"], wl["nx"]
        self.params = params_from_workload(wl, storage, phi_ref)
        nbytes = lb3_workspace_bytes(self.params)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.workspace.device)
        shape = (self.nz, self.ny, self.nx)
        self._phi0 = _f64(phi0, (self.m, *shape))
        self._u0 = _f64(u0, (3, *shape))
        self._p0 = None if p0 is None else _f64(p0, shape)
        h = C.c_void_p()
        _check(lib().lb3_init(C.byref(self.params), self.workspace.data_ptr(), nbytes, self.stream.cuda_stream,
                              self._phi0.ctypes.data, self._u0.ctypes.data,
                              None if self._p0 is None else self._p0.ctypes.data, C.byref(h)))
        self.handle = h

    def step(self, n: int):
        _check(lib().lb3_step(self.handle, int(n)))

    def moments(self):
        shape = (self.nz, self.ny, self.nx)
        phi = np.empty((self.m, *shape))
        u = np.empty((3, *shape))
        p = np.empty(shape)
        _check(lib().lb3_moments(self.handle, phi.ctypes.data, u.ctypes.data, p.ctypes.data))
        return phi, u, p

    def populations(self):
        shape = (self.nz, self.ny, self.nx)
        f = np.empty((self.m, 7, *shape))
        h = np.empty((19, *shape))
        _check(lib().lb3_populations(self.handle, f.ctypes.data, h.ctypes.data))
        return f, h

    def mass(self):
        out = np.empty(self.m + 1)
        _check(lib().lb3_mass(self.handle, out.ctypes.data))
        return out

    def set_tile(self, tx: int, ty: int):
        _check(lib().lb3_set_tile(self.handle, int(tx), int(ty)))

    @property
    def t(self) -> int:
        t = C.c_int64()
        _check(lib().lb3_time(self.handle, C.byref(t)))
        return t.value

    def close(self):
        if getattr(self, "handle", None) is not None:
            lib().lb3_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
