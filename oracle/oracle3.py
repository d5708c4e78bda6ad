"""Python wrapper of the plain FP64 CPU oracle of the 3-D model (``lb3_oracle.c``:
D3Q7 scalars, D3Q19 fluid).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark are the only callers.  The product library never imports
this module and this module never imports the product package.

Arrays: ``f[a][i][z][y][x]`` (7 per scalar), ``h[i][z][y][x]`` (19),
``Sold[a][z][y][x]``, ``phi[a][z][y][x]``, ``u[d][z][y][x]``, ``p[z][y][x]``;
lattice units (dx = dt = 1).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lb3_oracle.c")
LIB_OVERRIDE = os.environ.get("LB3_ORACLE_LIBRARY")
LIB = LIB_OVERRIDE or os.path.join(HERE, "liblb3oracle.so")
MAXM = 4

FLUID = {"periodic": 0, "noslip": 1}
SCALAR = {"periodic": 0, "noflux": 1, "dirichlet": 2}


class Orc3Cfg(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("m", C.c_int32),
        ("mutation", C.c_int32),
        ("fluid_bc", C.c_int32 * 6),
        ("scalar_bc", (C.c_int32 * MAXM) * 6),
        ("pad_", C.c_int32),
        ("tau_f", C.c_double), ("rho0", C.c_double),
        ("D", C.c_double * (MAXM * MAXM)),
        ("K", C.c_double * (MAXM * MAXM)),
        ("F0", C.c_double * 3),
        ("Fphi", C.c_double * (MAXM * 3)),
        ("wall", C.c_double * (6 * MAXM)),
    ]


def build(force: bool = False, openmp: bool = True) -> str:
    """Compile with gcc (plain -O2, no fast-math, no FMA contraction)."""
    if LIB_OVERRIDE:
        return LIB
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math"]
    if openmp:
        cmd.append("-fopenmp")
    cmd += [SRC, "-o", LIB + ".tmp", "-lm"]
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB)
        dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
        L.orc3_cfg_size.restype = C.c_size_t
        L.orc3_init.argtypes = [C.POINTER(Orc3Cfg), dp, dp, C.c_void_p, dp, dp, dp]
        L.orc3_step.argtypes = [C.POINTER(Orc3Cfg), dp, dp, dp, C.c_int64]
        L.orc3_moments.argtypes = [C.POINTER(Orc3Cfg), dp, dp, dp, dp, dp]
        L.orc3_feq.argtypes = [C.c_int, dp, dp, dp]
        L.orc3_feq.restype = None
        L.orc3_heq.argtypes = [C.c_double, dp, C.c_double, dp]
        L.orc3_heq.restype = None
        L.orc3_force_pop.argtypes = [dp, dp]
        L.orc3_force_pop.restype = None
        L.orc3_aux_source.argtypes = [C.c_int, dp, dp, dp, dp, dp, dp]
        L.orc3_aux_source.restype = None
        L.orc3_relaxation_matrix.argtypes = [C.c_int, dp, dp]
        assert L.orc3_cfg_size() == C.sizeof(Orc3Cfg), "oracle record layout mismatch"
        _lib = L
    return _lib


def make_cfg(wl: dict, mutation: int = 0) -> Orc3Cfg:
    c = Orc3Cfg()
    m = wl["m"]
    c.nx, c.ny, c.nz, c.m = wl["nx"], wl["ny"], wl["nz"], m
    c.mutation = mutation
    fb = wl.get("fluid_bc", ["periodic"] * 6)
    sb = wl.get("scalar_bc", [["periodic"] * m] * 6)
    for s in range(6):
        c.fluid_bc[s] = FLUID[fb[s]]
        for a in range(m):
            c.scalar_bc[s][a] = SCALAR[sb[s][a]]
    c.tau_f = wl["tau_f"]
    c.rho0 = wl.get("rho0", 1.0)
    D = np.asarray(wl["D"], dtype=np.float64).reshape(m, m)
    K = np.asarray(wl.get("K", np.zeros((m, m))), dtype=np.float64).reshape(m, m)
    for a in range(m):
        for b in range(m):
            c.D[a * m + b] = D[a, b]
            c.K[a * m + b] = K[a, b]
    F0 = wl.get("F0", [0.0, 0.0, 0.0])
    for d in range(3):
        c.F0[d] = F0[d]
    Fphi = np.asarray(wl.get("Fphi", np.zeros((m, 3))), dtype=np.float64).reshape(m, 3)
    for a in range(m):
        for d in range(3):
            c.Fphi[3 * a + d] = Fphi[a, d]
    wall = np.asarray(wl.get("wall", np.zeros((6, m))), dtype=np.float64).reshape(6, m)
    for s in range(6):
        for a in range(m):
            c.wall[s * MAXM + a] = wall[s, a]
    return c


class Oracle3:
    """Stateful convenience around orc3_init / orc3_step / orc3_moments."""

    def __init__(self, wl: dict, phi0, u0, p0=None, mutation: int = 0):
        self.L = lib()
        self.cfg = make_cfg(wl, mutation)
        nx, ny, nz, m = wl["nx"], wl["ny"], wl["nz"], wl["m"]
        self.shape = (nz, ny, nx)
        self.m = m
        self.f = np.zeros((m, 7, nz, ny, nx))
        self.h = np.zeros((19, nz, ny, nx))
        self.Sold = np.zeros((m, nz, ny, nx))
        phi0 = np.ascontiguousarray(phi0, dtype=np.float64).reshape(m, nz, ny, nx)
        u0 = np.ascontiguousarray(u0, dtype=np.float64).reshape(3, nz, ny, nx)
        self._p0 = None if p0 is None else np.ascontiguousarray(p0, dtype=np.float64).reshape(nz, ny, nx)
        pp = None if self._p0 is None else self._p0.ctypes.data_as(C.c_void_p)
        if self.L.orc3_init(C.byref(self.cfg), phi0, u0, pp, self.f, self.h, self.Sold) != 1:
            raise ValueError("oracle: bad configuration")
        self.t = 0

    def step(self, n: int):
        if self.L.orc3_step(C.byref(self.cfg), self.f, self.h, self.Sold, int(n)) != 1:
            raise RuntimeError("oracle step failed (singular relaxation matrix or no memory)")
        self.t += int(n)

    def moments(self):
        nz, ny, nx = self.shape
        phi = np.zeros((self.m, nz, ny, nx))
        u = np.zeros((3, nz, ny, nx))
        p = np.zeros((nz, ny, nx))
        self.L.orc3_moments(C.byref(self.cfg), self.f, self.h, phi, u, p)
        return phi, u, p


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64).ravel()


def feq(phi, u):
    m = len(phi)
    out = np.zeros(m * 7)
    lib().orc3_feq(m, _f64(phi), _f64(u), out)
    return out.reshape(m, 7)


def heq(p, u, rho0):
    out = np.zeros(19)
    lib().orc3_heq(float(p), _f64(u), float(rho0), out)
    return out


def force_pop(F):
    out = np.zeros(19)
    lib().orc3_force_pop(_f64(F), out)
    return out


def aux_source(omega, phi, S, u, F):
    m = len(phi)
    out = np.zeros(m * 7)
    lib().orc3_aux_source(m, _f64(omega), _f64(phi), _f64(S), _f64(u), _f64(F), out)
    return out.reshape(m, 7)


def relaxation_matrix(D):
    D = np.ascontiguousarray(D, dtype=np.float64)
    m = D.shape[0]
    out = np.zeros(m * m)
    assert lib().orc3_relaxation_matrix(m, D.ravel(), out) == 1
    return out.reshape(m, m)
