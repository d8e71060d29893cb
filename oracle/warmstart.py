"""Warm-start field mapping of the oracle (test infrastructure).

TEST INFRASTRUCTURE ONLY: the plain definition of what the library's warm
start computes before it sets equilibrium populations, written as loops over
nodes in float64.  Shares no code with the product path.

Given fields on an sx x sy cell-centred grid covering the cavity
(channel-last (u_x, u_y, theta, phi[, rho_f deviation]) after the affine map
a_c v + b_c):
  * lattice node (x, y) samples the source at the cell-centred coordinate
    s_x = (x + 1/2) sx / nx - 1/2 (likewise y), clamped to [0, sx - 1], by
    bilinear interpolation;
  * phi is clipped at 0 and rescaled so that its sum over the lattice equals
    the particle inventory of the cold start, sum max(phi0 + A xi, 0) (the
    particle mass of a closed cavity is conserved, so the steady state
    depends on it); a field with no particles left becomes uniform;
  * the fluid partial density is 1 - phi0 plus the density deviation less
    its lattice mean (the fluid mass is conserved as well).
"""
from __future__ import annotations

import math

import numpy as np


def _axis(n_dst: int, n_src: int, i: int):
    s = (i + 0.5) * n_src / n_dst - 0.5
    s = min(max(s, 0.0), n_src - 1.0)
    i0 = int(math.floor(s))
    i1 = min(i0 + 1, n_src - 1)
    return i0, i1, s - i0


def resample(fields: np.ndarray, nx: int, ny: int, scale=None, offset=None) -> np.ndarray:
    """fields: (sy, sx, nc).  Returns (nc, ny, nx) float64."""
    sy, sx, nc = fields.shape
    scale = [1.0] * nc if scale is None else list(scale)
    offset = [0.0] * nc if offset is None else list(offset)
    out = np.zeros((nc, ny, nx))
    for y in range(ny):
        y0, y1, wy = _axis(ny, sy, y)
        for x in range(nx):
            x0, x1, wx = _axis(nx, sx, x)
            for c in range(nc):
                v = lambda yy, xx: scale[c] * float(fields[yy, xx, c]) + offset[c]
                out[c, y, x] = ((1 - wy) * ((1 - wx) * v(y0, x0) + wx * v(y0, x1))
                                + wy * ((1 - wx) * v(y1, x0) + wx * v(y1, x1)))
    return out


def cold_inventory(phi0: float, amp: float, xi: np.ndarray | None, nn: int) -> float:
    if xi is None:
        return max(phi0, 0.0) * nn
    return float(sum(max(phi0 + amp * float(v), 0.0) for v in np.ravel(xi)))


def renormalize(phi: np.ndarray, inventory: float) -> np.ndarray:
    p = np.maximum(phi, 0.0)
    total = float(p.sum())
    if total > 0.0:
        return p * (inventory / total)
    return np.full_like(p, inventory / p.size)


def fluid_density(deviation: np.ndarray, phi0: float) -> np.ndarray:
    return (1.0 - phi0) + (deviation - deviation.mean())
