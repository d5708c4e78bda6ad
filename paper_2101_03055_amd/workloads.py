"""Seeded synthetic workloads: parameter records and initial fields.

This module holds no arithmetic of the lattice Boltzmann method itself: it only
draws seeded random numbers, lays out initial fields on the grid and converts
the paper's dimensionless parameters to lattice units (dx = dt = 1):

    D_lat = D dt*/dx*^2,  nu_lat = nu dt*/dx*^2,  F_lat = F dt*^2/dx*,
    S_lat = S dt*  (a source linear in phi scales its rate the same way),

where dx*, dt* are the dimensionless grid spacing and time step.  Both the
GPU library's binding and the CPU oracle's wrapper consume the same plain
``dict`` records and arrays produced here.

Record keys: nx, ny, m, model ('linear' | 'chemotaxis'), collision ('bgk' |
'mrt'), r_kind ('step' | 'smooth'), tau_f, rho0, mrt_s[9], D[m][m], K[m][m],
F0[2], Fphi[m][2], chi, beta, cstar, eps, fluid_bc[4], scalar_bc[4][m],
wall[4][m].  Sides are ordered x-, x+, y-, y+.  Fields are phi0[m][ny][nx],
u0[2][ny][nx], p0[ny][nx]; node (i, j) sits at the cell centre
((i + 1/2) dx, (j + 1/2) dx), so half-way walls lie on the domain edges.
"""
from __future__ import annotations

import math
import os

import numpy as np

def mrt_rates(tau_f, magic=3.0 / 16.0):
    """MRT rates tied to the viscous rate w = 1/tau_f.  The pressure scheme of
    the incompressible model (appendix A) rests on the BGK relaxation of the
    rest population h_0, which is made of the rho, e and eps moments only: they
    relax at w (as do the stress moments); the energy-flux moments q (zero on
    h_0) relax at the rate fixing (1/w - 1/2)(1/s_q - 1/2) = magic (3/16 makes
    half-way bounce-back exact for Poiseuille flow); j rates do not enter.
    Rates of rho, e or eps other than w (e.g. Lallemand & Luo's fixed 1.64,
    1.54, 1.9, or rho = 1) diverged in heated cavities and Taylor-Green flow."""
    w = 1.0 / tau_f
    sq = 1.0 / (magic / (1.0 / w - 0.5) + 0.5)
    return [w, w, w, 1.0, sq, 1.0, sq, w, w]


def _base(nx, ny, m, tau_f, D, **kw):
    wl = {
        "nx": int(nx), "ny": int(ny), "m": int(m), "model": "linear", "collision": "bgk",
        "r_kind": "step", "tau_f": float(tau_f), "rho0": 1.0, "mrt_s": mrt_rates(tau_f),
        "D": np.asarray(D, dtype=np.float64).reshape(m, m).tolist(),
        "K": np.zeros((m, m)).tolist(), "F0": [0.0, 0.0], "Fphi": np.zeros((m, 2)).tolist(),
        "chi": 0.0, "beta": 0.0, "cstar": 0.3, "eps": 0.0,
        "fluid_bc": ["periodic"] * 4, "scalar_bc": [["periodic"] * m for _ in range(4)],
        "wall": np.zeros((4, m)).tolist(),
    }
    wl.update(kw)
    return wl


def cell_centres(nx, ny):
    x = np.arange(nx) + 0.5
    y = np.arange(ny) + 0.5
    return np.meshgrid(x, y)  # X[j, i], Y[j, i]


# ---------------------------------------------------------------------------
# Plain-method case: Taylor-Green flow carrying two cross-diffusing Gaussian blobs
# ---------------------------------------------------------------------------
def taylor_green_blobs(n=64, seed=1, steps=1000, tau_f=0.8, U0=0.01, sigma=6.0,
                       D=((0.01, 0.002), (0.001, 0.01))):
    """Periodic n x n, D2Q9 BGK (tau_f), m = 2, constant D, no source, no force."""
    wl = _base(n, n, 2, tau_f, D)
    X, Y = cell_centres(n, n)
    k = 2.0 * math.pi / n
    u0 = np.stack([-U0 * np.cos(k * X) * np.sin(k * Y), U0 * np.sin(k * X) * np.cos(k * Y)])
    p0 = -(U0 * U0 / 4.0) * (np.cos(2 * k * X) + np.cos(2 * k * Y))
    rng = np.random.Generator(np.random.PCG64(seed))
    centres = rng.uniform(0.0, n, size=(2, 2))
    phi0 = np.empty((2, n, n))
    for a in range(2):
        dx = (X - centres[a, 0] + n / 2) % n - n / 2  # minimum image
        dy = (Y - centres[a, 1] + n / 2) % n - n / 2
        phi0[a] = 1.0 + np.exp(-(dx * dx + dy * dy) / (2 * sigma * sigma))
    wl["steps"] = steps
    wl["name"] = f"taylor_green_blobs_{n}x{n}"
    return wl, phi0, u0, p0


# ---------------------------------------------------------------------------
# Chemotaxis-fluid (Sec. 3.1): bacteria n, oxygen c
# ---------------------------------------------------------------------------
def chemotaxis(nx, ny, dx, dt, alpha, beta, delta, gamma, Sc, n0, c0=None,
               r_kind="step", cstar=0.3, eps=None, top_fluid="freeslip"):
    """Dimensionless chemotaxis-fluid system (Sec. 3.1) in lattice units.

    D = [[1, -alpha r(c) n], [0, delta]], S = (0, -beta r(c) n), nu = Sc,
    F = -Sc gamma n z.  Top: no flux of n, c = 1 (Dirichlet), free-slip fluid;
    bottom: no flux, no-slip; periodic in x.
    """
    s = dt / (dx * dx)
    wl = _base(nx, ny, 2, 3.0 * Sc * s + 0.5, [[1.0 * s, 0.0], [0.0, delta * s]])
    wl.update({
        "model": "chemotaxis", "chi": alpha * s, "beta": beta * dt, "cstar": cstar,
        "r_kind": r_kind, "eps": (dx if eps is None else eps),
        "Fphi": [[0.0, -Sc * gamma * dt * dt / dx], [0.0, 0.0]],
        "fluid_bc": ["periodic", "periodic", "noslip", top_fluid],
        "scalar_bc": [["periodic", "periodic"], ["periodic", "periodic"],
                      ["noflux", "noflux"], ["noflux", "dirichlet"]],
        "wall": [[0.0, 0.0], [0.0, 0.0], [0.0, 0.0], [0.0, 1.0]],
        "dx": dx, "dt": dt,
    })
    phi0 = np.empty((2, ny, nx))
    phi0[0] = n0
    phi0[1] = 1.0 if c0 is None else c0
    u0 = np.zeros((2, ny, nx))
    return wl, phi0, u0, np.zeros((ny, nx))


def chemotaxis_plume(nx=512, ny=256, seed=2, ratio=6.25e-4, alpha=10.0, beta=20.0, delta=5.0,
                     gamma=2000.0, Sc=500.0, amp=0.01):
    """Plume-formation workload (Sec. 3.1.3 parameters) on [-1, 1] x [0, 1].

    dx = 1/ny, dt = ratio dx^2 (the paper's dt/dx^2 of Sec. 3.1.1);
    n0 = 1 + amp U(-1, 1) (seeded), c0 = 1, u0 = 0.
    """
    dx = 1.0 / ny
    dt = ratio * dx * dx
    rng = np.random.Generator(np.random.PCG64(seed))
    n0 = 1.0 + amp * rng.uniform(-1.0, 1.0, size=(ny, nx))
    wl, phi0, u0, p0 = chemotaxis(nx, ny, dx, dt, alpha, beta, delta, gamma, Sc, n0)
    wl["name"] = f"chemotaxis_plume_{nx}x{ny}"
    return wl, phi0, u0, p0


def chemotaxis_sinusoidal(nx=300, ny=50, dt=2.5e-7, a=3.0, alpha=10.0, beta=10.0, delta=5.0, gamma=1000.0,
                          Sc=500.0):
    """Plumes from a sinusoidally modulated layer (Sec. 3.1.3, beta = 10,
    gamma = 1000) on [-a, a] x [0, 1], dx = 1/ny (nx = 2 a ny):
    n0 = 1 where y > 0.499 - 0.01 sin((x - 1.5) pi), 0.5 below; c0 = 1, u0 = 0
    (cell centres).  Deterministic: no random draw.  The defaults are the
    domain [-3, 3] x [0, 1], dx = 0.02 and dt = 2.5e-7 that the paper states
    for its chemotaxis runs (Secs. 3.1.1 and 3.1.3)."""
    dx = 1.0 / ny
    if abs(nx * dx - 2.0 * a) > 1e-9:
        raise ValueError("nx must equal 2 a ny")
    X, Y = cell_centres(nx, ny)
    x, y = -a + X * dx, Y * dx
    n0 = np.where(y > 0.499 - 0.01 * np.sin((x - 1.5) * math.pi), 1.0, 0.5)
    wl, phi0, u0, p0 = chemotaxis(nx, ny, dx, dt, alpha, beta, delta, gamma, Sc, n0)
    wl["name"] = f"chemotaxis_sinusoidal_{nx}x{ny}"
    return wl, phi0, u0, p0


def chemotaxis_layer(alpha, beta, delta, nx=100, ny=50, a=1.0, dt=1e-8, gamma=418.0, Sc=7700.0, cstar=0.3):
    """Parameter-influence case of Sec. 3.1.2 on [-a, a] x [0, 1], dx = 1/ny
    (nx = 2 a ny): n0 = 1 where y > 0.501 - 0.01 sin((x - 0.5) pi), 0.5 below;
    c0 = 1, u0 = 0 (cell centres); gamma = 418, Sc = 7700, dt = 1e-8 and the
    regularised cut-off r(c) with eps = dx.  Deterministic: no random draw.
    Defaults: dx = 0.02 (the grid the paper states for its chemotaxis runs)
    and one period of the modulation, x in [-1, 1]."""
    dx = 1.0 / ny
    if abs(nx * dx - 2.0 * a) > 1e-9:
        raise ValueError("nx must equal 2 a ny")
    X, Y = cell_centres(nx, ny)
    x, y = -a + X * dx, Y * dx
    n0 = np.where(y > 0.501 - 0.01 * np.sin((x - 0.5) * math.pi), 1.0, 0.5)
    wl, phi0, u0, p0 = chemotaxis(nx, ny, dx, dt, alpha, beta, delta, gamma, Sc, n0, r_kind="smooth",
                                  cstar=cstar, eps=dx)
    wl["name"] = f"chemotaxis_layer_a{alpha:g}_b{beta:g}_d{delta:g}_{nx}x{ny}"
    return wl, phi0, u0, p0


def chemotaxis_steady(ny=50, nx=4, ratio=0.01, alpha=10.0, beta=10.0, delta=5.0, gamma=1000.0,
                      Sc=500.0):
    """Steady validation case of Sec. 3.1.1: n0 = pi/40, c0 = 1, u0 = 0 on a
    strip of the x-homogeneous domain (periodic in x), dx = 1/ny."""
    dx = 1.0 / ny
    dt = ratio * dx * dx
    n0 = np.full((ny, nx), math.pi / 40.0)
    wl, phi0, u0, p0 = chemotaxis(nx, ny, dx, dt, alpha, beta, delta, gamma, Sc, n0)
    wl["name"] = f"chemotaxis_steady_{nx}x{ny}"
    return wl, phi0, u0, p0


# ---------------------------------------------------------------------------
# Double-diffusive convection with Soret and Dufour effects (Sec. 3.2)
# ---------------------------------------------------------------------------
def ddc(L, Ra, Pr, Le, Nc, Sr, Df, A=1.0, u_lat=0.05, collision="bgk"):
    """Dimensionless DDC cavity [0, 1] x [0, A] on L x round(A L) nodes.

    D = [[1, Df], [Sr/Le, 1/Le]], nu = Pr, F = Ra Pr (T + Nc C) z, S = 0.
    T = C = 1 at x = 0 and 0 at x = 1 (Dirichlet), no flux on y walls, no-slip
    everywhere; T = C = u = 0 at t = 0.  dt* is fixed by the lattice velocity
    scale sqrt(Ra Pr) dt*/dx* = u_lat.
    """
    nx, ny = int(L), int(round(A * L))
    dx = 1.0 / L
    dt = u_lat * dx / math.sqrt(Ra * Pr)
    s = dt / (dx * dx)
    D = np.array([[1.0, Df], [Sr / Le, 1.0 / Le]]) * s
    g = Ra * Pr * dt * dt / dx
    wl = _base(nx, ny, 2, 3.0 * Pr * s + 0.5, D)
    wl.update({
        "collision": collision,
        "Fphi": [[0.0, g], [0.0, g * Nc]],
        "fluid_bc": ["noslip"] * 4,
        "scalar_bc": [["dirichlet", "dirichlet"], ["dirichlet", "dirichlet"],
                      ["noflux", "noflux"], ["noflux", "noflux"]],
        "wall": [[1.0, 1.0], [0.0, 0.0], [0.0, 0.0], [0.0, 0.0]],
        "dx": dx, "dt": dt, "Ra": Ra, "Pr": Pr, "Le": Le, "Nc": Nc, "Sr": Sr, "Df": Df,
        "A": A, "u_lat": u_lat,
        "name": f"ddc_{nx}x{ny}_Ra{Ra:g}",
    })
    phi0 = np.zeros((2, ny, nx))
    u0 = np.zeros((2, ny, nx))
    return wl, phi0, u0, np.zeros((ny, nx))


def ddc_cavity(L=256):
    """Double-diffusive cavity with Soret/Dufour: Ra 1e5, Pr 0.71, Le 2, N 1, Sr = Df = 0.1."""
    return ddc(L, Ra=1e5, Pr=0.71, Le=2.0, Nc=1.0, Sr=0.1, Df=0.1)


def sweep_params(count=256, seed=4, sizes=None):
    """Parameter law of the batched sweep: L uniform over {64, 96, ..., 256},
    Ra log-uniform in [1e3, 1e6], Le U[1, 5], Nc U[-2, 2], Sr, Df U[0, 0.5], Pr 0.71."""
    rng = np.random.Generator(np.random.PCG64(seed))
    choices = np.arange(64, 257, 32) if sizes is None else np.asarray(sizes)
    out = []
    for _ in range(count):
        out.append({
            "L": int(rng.choice(choices)),
            "Ra": float(10.0 ** rng.uniform(3.0, 6.0)),
            "Le": float(rng.uniform(1.0, 5.0)),
            "Nc": float(rng.uniform(-2.0, 2.0)),
            "Sr": float(rng.uniform(0.0, 0.5)),
            "Df": float(rng.uniform(0.0, 0.5)),
            "Pr": 0.71,
        })
    return out


# ---------------------------------------------------------------------------
# Generic seeded cases for parity tests (exercise every boundary kind)
# ---------------------------------------------------------------------------
def random_case(nx, ny, m=2, seed=0, fluid_bc=None, scalar_bc=None, model="linear",
                collision="bgk", force=True, source=False, amp=0.05):
    """A small random case: smooth-ish random fields, random SPD-dominant D."""
    rng = np.random.Generator(np.random.PCG64(seed))
    D = np.diag(rng.uniform(0.02, 0.2, size=m))
    D += 0.2 * np.min(np.diag(D)) * rng.uniform(-1, 1, size=(m, m)) * (1 - np.eye(m))
    wl = _base(nx, ny, m, float(rng.uniform(0.6, 1.2)), D, collision=collision)
    if fluid_bc is not None:
        wl["fluid_bc"] = list(fluid_bc)
    if scalar_bc is not None:
        wl["scalar_bc"] = [list(r) for r in scalar_bc]
    wl["wall"] = rng.uniform(0.5, 1.5, size=(4, m)).tolist()
    if force:
        wl["F0"] = rng.uniform(-1e-5, 1e-5, size=2).tolist()
        wl["Fphi"] = rng.uniform(-1e-5, 1e-5, size=(m, 2)).tolist()
    if source:
        wl["K"] = (-rng.uniform(0.0, 2e-3, size=(m, m))).tolist()
    if model == "chemotaxis":
        wl.update({"model": "chemotaxis", "chi": float(rng.uniform(0.005, 0.02)),
                   "beta": float(rng.uniform(1e-4, 1e-3)), "cstar": 0.95})
        wl["D"] = [[float(D[0, 0]), 0.0], [0.0, float(D[1, 1])]]
    phi0 = 1.0 + amp * rng.standard_normal(size=(m, ny, nx))
    u0 = 0.02 * rng.standard_normal(size=(2, ny, nx))
    p0 = 1e-3 * rng.standard_normal(size=(ny, nx))
    wl["name"] = f"random_{nx}x{ny}_s{seed}"
    return wl, phi0, u0, p0


# ---------------------------------------------------------------------------
# Case 1 (no fluid): species carried by a prescribed velocity field
# ---------------------------------------------------------------------------
def cde_case(nx, ny, m=2, seed=0, walls=False, source=False, U=0.05):
    """Cross-diffusing species in a prescribed, divergence-free cellular flow
    u = U (sin(2 pi x/nx) cos(2 pi y/ny) ny/nx, -cos(2 pi x/nx) sin(2 pi y/ny))
    (the stream function U ny/(2 pi) sin sin, sampled at cell centres).
    walls: Dirichlet at x = 0 / nx, no flux at y = 0 / ny (the normal velocity
    vanishes on the y walls); otherwise periodic."""
    rng = np.random.Generator(np.random.PCG64(seed))
    D = np.diag(rng.uniform(0.03, 0.12, size=m))
    D += 0.2 * np.min(np.diag(D)) * rng.uniform(-1, 1, size=(m, m)) * (1 - np.eye(m))
    wl = _base(nx, ny, m, 0.8, D, model="cde")
    if walls:
        wl["fluid_bc"] = ["noslip", "noslip", "noslip", "noslip"]
        wl["scalar_bc"] = [["dirichlet"] * m, ["dirichlet"] * m, ["noflux"] * m, ["noflux"] * m]
        wl["wall"] = rng.uniform(0.5, 1.5, size=(4, m)).tolist()
    if source:
        wl["K"] = (-rng.uniform(0.0, 2e-3, size=(m, m))).tolist()
    X, Y = cell_centres(nx, ny)
    kx, ky = 2 * np.pi * X / nx, 2 * np.pi * Y / ny
    u0 = U * np.stack([np.sin(kx) * np.cos(ky) * ny / nx, -np.cos(kx) * np.sin(ky)])
    phi0 = 1.0 + 0.05 * rng.standard_normal(size=(m, ny, nx))
    wl["name"] = f"cde_{nx}x{ny}_s{seed}"
    return wl, phi0, u0, None


# ---------------------------------------------------------------------------
# Surrogate data: one seed per cavity, the sweep's parameter law
# ---------------------------------------------------------------------------
def sweep_case(seed, L=128):
    """Parameters of one cavity drawn with its own seed (sweep law, fixed L)."""
    d = sweep_params(1, seed=seed, sizes=[L])[0]
    d["seed"] = int(seed)
    return d


def normalise(pd):
    """The surrogate's five inputs in [0, 1]: log10 Ra, Le, Nc, Sr, Df over the law's ranges."""
    return [(np.log10(pd["Ra"]) - 3.0) / 3.0, (pd["Le"] - 1.0) / 4.0, (pd["Nc"] + 2.0) / 4.0,
            pd["Sr"] / 0.5, pd["Df"] / 0.5]


def ddc_case(pd, collision="bgk", u_lat=0.1):
    """Cavity workload (record, cold initial fields) for one parameter draw."""
    return ddc(pd["L"], Ra=pd["Ra"], Pr=pd.get("Pr", 0.71), Le=pd["Le"], Nc=pd["Nc"], Sr=pd["Sr"], Df=pd["Df"],
               u_lat=u_lat, collision=collision)


# ---------------------------------------------------------------------------
# Three dimensions (D3Q7 scalars, D3Q19 fluid): records carry nz, 6 sides
# (x-, x+, y-, y+, z-, z+), F0[3], Fphi[m][3]; fields phi0[m][nz][ny][nx],
# u0[3][nz][ny][nx], p0[nz][ny][nx]
# ---------------------------------------------------------------------------
def base3(nx, ny, nz, m, tau_f, D, **kw):
    wl = {
        "dim": 3, "nx": int(nx), "ny": int(ny), "nz": int(nz), "m": int(m), "tau_f": float(tau_f), "rho0": 1.0,
        "D": np.asarray(D, dtype=np.float64).reshape(m, m).tolist(), "K": np.zeros((m, m)).tolist(),
        "F0": [0.0, 0.0, 0.0], "Fphi": np.zeros((m, 3)).tolist(),
        "fluid_bc": ["periodic"] * 6, "scalar_bc": [["periodic"] * m for _ in range(6)],
        "wall": np.zeros((6, m)).tolist(),
    }
    wl.update(kw)
    return wl


def cell_centres3(nx, ny, nz):
    """X, Y, Z of the cell centres, each shaped [nz][ny][nx]."""
    z, y, x = np.meshgrid(np.arange(nz) + 0.5, np.arange(ny) + 0.5, np.arange(nx) + 0.5, indexing="ij")
    return x, y, z


def random_case3(nx, ny, nz, m=2, seed=0, fluid_bc=None, scalar_bc=None, force=True, source=False, amp=0.05):
    """A small random 3-D case: smooth-ish random fields, SPD-dominant D."""
    rng = np.random.Generator(np.random.PCG64(seed))
    D = np.diag(rng.uniform(0.02, 0.15, size=m))
    D += 0.2 * np.min(np.diag(D)) * rng.uniform(-1, 1, size=(m, m)) * (1 - np.eye(m))
    wl = base3(nx, ny, nz, m, float(rng.uniform(0.6, 1.2)), D)
    if fluid_bc is not None:
        wl["fluid_bc"] = list(fluid_bc)
    if scalar_bc is not None:
        wl["scalar_bc"] = [list(r) for r in scalar_bc]
    wl["wall"] = rng.uniform(0.5, 1.5, size=(6, m)).tolist()
    if force:
        wl["F0"] = rng.uniform(-2e-5, 2e-5, size=3).tolist()
        wl["Fphi"] = rng.uniform(-2e-5, 2e-5, size=(m, 3)).tolist()
    if source:
        wl["K"] = (-rng.uniform(0.0, 2e-3, size=(m, m))).tolist()
    shape = (nz, ny, nx)

    def smooth(a):  # cheap periodic smoothing so the fields are not pure noise
        for ax in (-1, -2, -3):
            a = 0.25 * (np.roll(a, 1, ax) + 2 * a + np.roll(a, -1, ax))
        return a

    phi0 = 1.0 + amp * np.stack([smooth(rng.standard_normal(shape)) for _ in range(m)])
    u0 = 0.02 * np.stack([smooth(rng.standard_normal(shape)) for _ in range(3)])
    p0 = 1e-3 * smooth(rng.standard_normal(shape))
    wl["name"] = f"random3_{nx}x{ny}x{nz}_s{seed}"
    return wl, phi0, u0, p0


def taylor_green3(n=256, m=2, seed=1, tau_f=0.8, U0=0.02, sigma=None, D=((0.01, 0.002), (0.001, 0.01))):
    """Periodic n^3 box: the 3-D Taylor-Green vortex
    u = U0 sin kx cos ky cos kz, v = -U0 cos kx sin ky cos kz, w = 0,
    p0 = (U0^2/16)(cos 2kx + cos 2ky)(cos 2kz + 2), carrying m cross-diffusing
    Gaussian blobs (centres drawn with the seed, minimum image)."""
    sigma = n / 10.0 if sigma is None else sigma
    D = np.asarray(D, dtype=np.float64)[:m, :m]
    wl = base3(n, n, n, m, tau_f, D)
    X, Y, Z = cell_centres3(n, n, n)
    k = 2.0 * math.pi / n
    u0 = np.stack([U0 * np.sin(k * X) * np.cos(k * Y) * np.cos(k * Z),
                   -U0 * np.cos(k * X) * np.sin(k * Y) * np.cos(k * Z),
                   np.zeros_like(X)])
    p0 = (U0 * U0 / 16.0) * (np.cos(2 * k * X) + np.cos(2 * k * Y)) * (np.cos(2 * k * Z) + 2.0)
    rng = np.random.Generator(np.random.PCG64(seed))
    centres = rng.uniform(0.0, n, size=(m, 3))
    phi0 = np.empty((m, n, n, n))
    for a in range(m):
        d2 = np.zeros_like(X)
        for c, C_ in zip((X, Y, Z), centres[a]):
            dd = (c - C_ + n / 2) % n - n / 2
            d2 += dd * dd
        phi0[a] = 1.0 + np.exp(-d2 / (2 * sigma * sigma))
    wl["name"] = f"taylor_green3_{n}^3"
    return wl, phi0, u0, p0


# ---------------------------------------------------------------------------
# Named configurations (JSON files in configs/): each names a generator of
# this module, its arguments and the run settings
# ---------------------------------------------------------------------------
CONFIG_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "configs")


def config_names():
    return sorted(f[:-5] for f in os.listdir(CONFIG_DIR) if f.endswith(".json"))


def load_config(name: str):
    """(config dict, cases): cases is a list of (record, phi0, u0, p0) for the
    generators that build fields, or of parameter draws for the surrogate's
    seed ranges (built cavity by cavity by its study)."""
    import json

    path = name if name.endswith(".json") else os.path.join(CONFIG_DIR, name + ".json")
    with open(path) as fh:
        cfg = json.load(fh)
    gen, kw = cfg["workload"], cfg.get("kwargs", {})
    if gen == "sweep":
        cases = [ddc_case(pd) for pd in sweep_params(**kw)]
    elif gen == "sweep_case":
        lo, hi = cfg["seeds"]["test"]
        cases = [sweep_case(s, **kw) for s in range(lo, hi)]
    else:
        cases = [globals()[gen](**kw)]
    return cfg, cases
