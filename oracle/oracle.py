"""Python wrapper of the plain FP64 CPU oracle (``lb_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark are the only callers.  The product library never imports
this module and this module never imports the product package.

Arrays use the layout the C oracle documents: ``f[a][i][y][x]`` for the m D2Q5
scalar lattices, ``h[i][y][x]`` for the D2Q9 fluid lattice, ``Sold[a][y][x]``
for the previous-step source, ``phi[a][y][x]``, ``u[d][y][x]`` and ``p[y][x]``.
All values are in lattice units (dx = dt = 1).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lb_oracle.c")
# LB_ORACLE_LIBRARY selects a prebuilt copy (the sanitized build of the
# sanitizer test); it is then used as is, never rebuilt
LIB_OVERRIDE = os.environ.get("LB_ORACLE_LIBRARY")
LIB = LIB_OVERRIDE or os.path.join(HERE, "liblboracle.so")
MAXM = 4

# codes used by the oracle's record (its own; the GPU library has its own)
FLUID = {"periodic": 0, "noslip": 1, "freeslip": 2}
SCALAR = {"periodic": 0, "noflux": 1, "dirichlet": 2}
MODEL = {"linear": 0, "chemotaxis": 1, "cde": 2}


class OrcCfg(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("m", C.c_int32),
        ("model", C.c_int32), ("collision", C.c_int32), ("r_kind", C.c_int32),
        ("mutation", C.c_int32),
        ("fluid_bc", C.c_int32 * 4),
        ("scalar_bc", (C.c_int32 * MAXM) * 4),
        ("pad_", C.c_int32),
        ("tau_f", C.c_double), ("rho0", C.c_double),
        ("mrt_s", C.c_double * 9),
        ("D", C.c_double * (MAXM * MAXM)),
        ("F0", C.c_double * 2),
        ("Fphi", C.c_double * (MAXM * 2)),
        ("K", C.c_double * (MAXM * MAXM)),
        ("chi", C.c_double), ("beta", C.c_double), ("cstar", C.c_double), ("eps", C.c_double),
        ("wall", C.c_double * (4 * MAXM)),
        ("lam", C.c_double * (MAXM * MAXM)),
        ("varphi", C.c_double),
        ("gamma", C.c_double * MAXM),
    ]


def build(force: bool = False, openmp: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math, no FMA contraction)."""
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
        L.orc_cfg_size.restype = C.c_size_t
        L.orc_init.argtypes = [C.POINTER(OrcCfg), dp, dp, C.c_void_p, dp, dp, dp]
        L.orc_step.argtypes = [C.POINTER(OrcCfg), dp, dp, dp, C.c_int64]
        L.orc_moments.argtypes = [C.POINTER(OrcCfg), dp, dp, dp, dp, dp]
        L.orc_feq.argtypes = [C.c_int, dp, dp, dp, dp]
        L.orc_feq.restype = None
        L.orc_heq.argtypes = [C.c_double, dp, C.c_double, dp]
        L.orc_heq.restype = None
        L.orc_force_pop.argtypes = [dp, dp, C.c_double, dp]
        L.orc_force_pop.restype = None
        L.orc_aux_source.argtypes = [C.c_int, dp, dp, dp, dp, dp, dp]
        L.orc_aux_source.restype = None
        L.orc_source_pop.argtypes = [C.c_int, dp, dp]
        L.orc_source_pop.restype = None
        L.orc_relaxation_matrix.argtypes = [C.c_int, dp, dp, dp]
        L.orc_mrt_basis.argtypes = [dp, dp]
        L.orc_threads.restype = C.c_int
        L.orc_cutoff.argtypes = [C.POINTER(OrcCfg), C.c_double]
        L.orc_cutoff.restype = C.c_double
        assert L.orc_cfg_size() == C.sizeof(OrcCfg), "oracle record layout mismatch"
        _lib = L
    return _lib


def make_cfg(wl: dict, mutation: int = 0) -> OrcCfg:
    """Fill the oracle's record from a workload description (plain dict)."""
    c = OrcCfg()
    c.nx, c.ny, c.m = wl["nx"], wl["ny"], wl["m"]
    c.model = MODEL[wl.get("model", "linear")]
    c.collision = 1 if wl.get("collision", "bgk") == "mrt" else 0
    c.r_kind = 1 if wl.get("r_kind", "step") == "smooth" else 0
    c.mutation = mutation
    fb = wl.get("fluid_bc", ["periodic"] * 4)
    for s in range(4):
        c.fluid_bc[s] = FLUID[fb[s]]
    sb = wl.get("scalar_bc", [["periodic"] * wl["m"]] * 4)
    for s in range(4):
        for a in range(wl["m"]):
            c.scalar_bc[s][a] = SCALAR[sb[s][a]]
    c.tau_f = wl["tau_f"]
    c.rho0 = wl.get("rho0", 1.0)
    rates = wl.get("mrt_s", [1.0] * 9)
    for k in range(9):
        c.mrt_s[k] = rates[k]
    m = wl["m"]
    D = np.asarray(wl["D"], dtype=np.float64).reshape(m, m)
    K = np.asarray(wl.get("K", np.zeros((m, m))), dtype=np.float64).reshape(m, m)
    for a in range(m):
        for b in range(m):
            c.D[a * m + b] = D[a, b]
            c.K[a * m + b] = K[a, b]
    F0 = wl.get("F0", [0.0, 0.0])
    c.F0[0], c.F0[1] = F0
    Fphi = np.asarray(wl.get("Fphi", np.zeros((m, 2))), dtype=np.float64).reshape(m, 2)
    for a in range(m):
        c.Fphi[2 * a], c.Fphi[2 * a + 1] = Fphi[a]
    c.chi = wl.get("chi", 0.0)
    c.beta = wl.get("beta", 0.0)
    c.cstar = wl.get("cstar", 0.3)
    c.eps = wl.get("eps", 0.0)
    wall = np.asarray(wl.get("wall", np.zeros((4, m))), dtype=np.float64).reshape(4, m)
    for s in range(4):
        for a in range(m):
            c.wall[s * MAXM + a] = wall[s, a]
    lam = np.asarray(wl.get("lam", np.eye(m)), dtype=np.float64).reshape(m, m)
    for a in range(m):
        for b in range(m):
            c.lam[a * m + b] = lam[a, b]
    c.varphi = wl.get("varphi", 0.0)
    gam = wl.get("gamma_s", [0.0] * m)
    for a in range(m):
        c.gamma[a] = gam[a]
    return c


class Oracle:
    """Stateful convenience around the oracle's init/step/moments entry points."""

    def __init__(self, wl: dict, phi0, u0, p0=None, mutation: int = 0):
        self.L = lib()
        self.cfg = make_cfg(wl, mutation)
        nx, ny, m = wl["nx"], wl["ny"], wl["m"]
        self.shape = (ny, nx)
        self.m = m
        self.f = np.zeros((m, 5, ny, nx))
        self.h = np.zeros((9, ny, nx))
        self.Sold = np.zeros((m, ny, nx))
        phi0 = np.ascontiguousarray(phi0, dtype=np.float64).reshape(m, ny, nx)
        u0 = np.ascontiguousarray(u0, dtype=np.float64).reshape(2, ny, nx)
        self._p0 = None if p0 is None else np.ascontiguousarray(p0, dtype=np.float64).reshape(ny, nx)
        pp = None if self._p0 is None else self._p0.ctypes.data_as(C.c_void_p)
        ok = self.L.orc_init(C.byref(self.cfg), phi0, u0, pp, self.f, self.h, self.Sold)
        if ok != 1:
            raise ValueError("oracle: unsupported configuration (varphi != 0 needs BGK)")
        self.t = 0

    def step(self, n: int):
        ok = self.L.orc_step(C.byref(self.cfg), self.f, self.h, self.Sold, int(n))
        if ok != 1:
            raise RuntimeError("oracle step failed (singular relaxation matrix or no memory)")
        self.t += int(n)

    def moments(self):
        ny, nx = self.shape
        phi = np.zeros((self.m, ny, nx))
        u = np.zeros((2, ny, nx))
        p = np.zeros((ny, nx))
        self.L.orc_moments(C.byref(self.cfg), self.f, self.h, phi, u, p)
        return phi, u, p


# ---- single-node functions (for the moment-identity pins) -------------------
def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64).ravel()


def feq(phi, u, lam=None):
    """Eq. feq-phi (vartheta = 0); lam defaults to the identity."""
    m = len(phi)
    lam = np.eye(m) if lam is None else lam
    out = np.zeros(m * 5)
    lib().orc_feq(m, _f64(lam), _f64(phi), _f64(u), out)
    return out.reshape(m, 5)


def heq(p, u, rho0):
    out = np.zeros(9)
    lib().orc_heq(float(p), np.ascontiguousarray(u, dtype=np.float64), float(rho0), out)
    return out


def force_pop(F, u=(0.0, 0.0), varphi=0.0):
    """Eq. force at velocity u with the parameter varphi."""
    out = np.zeros(9)
    lib().orc_force_pop(_f64(F), _f64(u), float(varphi), out)
    return out


def aux_source(omega, phi, S, u, F):
    m = len(phi)
    out = np.zeros(m * 5)
    f64 = lambda a: np.ascontiguousarray(a, dtype=np.float64).ravel()
    lib().orc_aux_source(m, f64(omega), f64(phi), f64(S), f64(u), f64(F), out)
    return out.reshape(m, 5)


def source_pop(S):
    m = len(S)
    out = np.zeros(m * 5)
    lib().orc_source_pop(m, np.ascontiguousarray(S, dtype=np.float64), out)
    return out.reshape(m, 5)


def relaxation_matrix(D, lam=None):
    """Eq. omega-D; lam defaults to the identity."""
    D = np.ascontiguousarray(D, dtype=np.float64)
    m = D.shape[0]
    lam = np.eye(m) if lam is None else lam
    out = np.zeros(m * m)
    assert lib().orc_relaxation_matrix(m, D.ravel(), _f64(lam), out) == 1
    return out.reshape(m, m)


def mrt_basis():
    M = np.zeros(81)
    Mi = np.zeros(81)
    assert lib().orc_mrt_basis(M, Mi) == 1
    return M.reshape(9, 9), Mi.reshape(9, 9)


def cutoff(wl: dict, c: float) -> float:
    """r(c) of the workload's cut-off (step or regularised)."""
    cfg = make_cfg(wl)
    return float(lib().orc_cutoff(C.byref(cfg), float(c)))


def threads() -> int:
    return int(lib().orc_threads())


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))
