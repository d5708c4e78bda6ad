"""Oracle of the wall-flux diagnostics (Sec. 3.2, the Nusselt and Sherwood numbers).

Test infrastructure: only tests, the smoke check and the benchmark's CPU
baseline use it.  Plain numpy written from the definitions:

  Nu(y) = dT/dx + D_CT dC/dx,  Sh(y) = S_TC dT/dx + dC/dx  at the hot wall x = 0,

taken with the sign that makes the heat and solute flux into the cavity
positive, averaged over the wall.  For a general diffusion matrix this is row a
of -D grad(phi) . n divided by D_aa: row 0 of D = [[1, D_CT], [S_TC/Le, 1/Le]]
gives Nu and row 1 (times Le) gives Sh.

The paper asks for second-order one-sided ("upwind") differences.  With the
half-way walls used here the wall value sits half a spacing before the first
node, so the derivative is that of the quadratic through (0, phi_w),
(1/2, phi_0), (3/2, phi_1): (-8 phi_w + 9 phi_0 - phi_1) / 3 per spacing.
Lengths are scaled by the cavity depth across the wall (nodes x spacing = 1).
"""
from __future__ import annotations

import numpy as np


def normal_derivative(phi: np.ndarray, wall: float, side: int) -> np.ndarray:
    """d phi / dn along the inward normal of wall `side` (0: x=0, 1: x=nx,
    2: y=0, 3: y=ny) per unit cavity length, one value per wall node.
    phi has shape (ny, nx)."""
    ny, nx = phi.shape
    if side == 0:
        p0, p1, depth = phi[:, 0], phi[:, 1], nx
    elif side == 1:
        p0, p1, depth = phi[:, -1], phi[:, -2], nx
    elif side == 2:
        p0, p1, depth = phi[0, :], phi[1, :], ny
    elif side == 3:
        p0, p1, depth = phi[-1, :], phi[-2, :], ny
    else:
        raise ValueError("side must be 0..3")
    return (-8.0 * wall + 9.0 * p0 - p1) / 3.0 * depth


def wall_flux(phi: np.ndarray, D: np.ndarray, wall, side: int) -> np.ndarray:
    """Mean over the wall of -(1/D_aa) sum_b D_ab dphi_b/dn, for every species a.
    phi: (m, ny, nx) fields; D: (m, m); wall: the m Dirichlet values."""
    m = phi.shape[0]
    D = np.asarray(D, dtype=np.float64).reshape(m, m)
    g = np.stack([normal_derivative(phi[b], float(wall[b]), side) for b in range(m)])  # (m, len)
    out = np.empty(m)
    for a in range(m):
        out[a] = -np.mean(sum(D[a, b] * g[b] for b in range(m))) / D[a, a]
    return out
