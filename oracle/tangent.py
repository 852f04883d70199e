"""Tangent-linear maps of the 1D-1V step's stages, plain FP64 numpy.

TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT: only the tests may import this
module.  It shares nothing with the GPU library.

Each function is the exact derivative of one stage of the oracle's step along
a given direction, written from that stage's definition (the same grid
conventions as avl_oracle.c: cell-centred grids, cloud-in-cell weights one
cell wide, x periodic, velocity corners outside the grid dropped):

  push (Sec. 2, unmagnetised, kick then drift):
      E(x) = (1 - a) E_{i0} + a E_{i0+1},  a = x/dx - 1/2 - i0,
      v' = v + c E(x),  c = (q/m) dt kick,   x' = x + v' dt;
  reconstruction and moments (Eq. (reconstruction); rho of Sec. 2):
      N_g = sum_l alpha_gl f_l,  D_g = sum_l alpha_gl,  f_g = N_g / D_g,
      rho_i = q dv sum_j f_{j,i};
  field (Eq. (poissonk)): E = P rho is linear, so its tangent is the solve
      itself (``oracle.poisson``).

The reverse stages of the library are checked against these with the
dot-product identity <J du, lam> = <du, J^T lam>.  Within one cell the push is
linear and the reconstruction rational in the marker coordinates; the maps
hold wherever no marker sits exactly on a cell-centre line.
"""
from __future__ import annotations

import numpy as np

from . import Grid, poisson, reconstruct


def _axis(coord, lo, h):
    t = (coord - lo) / h - 0.5
    low = np.floor(t)
    return low.astype(np.int64), t - low


def push_tangent(grid: Grid, x, v, E, kick, dx, dv, dE):
    """(dx', dv') of the unmagnetised 1D-1V push at (x, v, E) along (dx, dv, dE)."""
    assert grid.vdim == 1
    x, v, E = (np.asarray(a, dtype=np.float64).reshape(-1) for a in (x, v, E))
    dx, dv, dE = (np.asarray(a, dtype=np.float64).reshape(-1) for a in (dx, dv, dE))
    h = grid.L / grid.nx
    i0, a = _axis(x, 0.0, h)
    ia = np.mod(i0, grid.nx)
    ib = np.mod(i0 + 1, grid.nx)
    c = grid.q / grid.m * grid.dt * kick
    da = dx / h
    dEl = (E[ib] - E[ia]) * da + (1.0 - a) * dE[ia] + a * dE[ib]
    dv1 = dv + c * dEl
    dx1 = dx + dv1 * grid.dt
    return dx1, dv1


def deposit_tangent(grid: Grid, x, v, f, dx, dv, df):
    """d rho (nx) of reconstruction + moments at markers (x, v, f) along
    (dx, dv, df); cells with D = 0 stay at f = 0 and carry nothing."""
    assert grid.vdim == 1
    x, v, f = (np.asarray(a, dtype=np.float64).reshape(-1) for a in (x, v, f))
    dx, dv, df = (np.asarray(a, dtype=np.float64).reshape(-1) for a in (dx, dv, df))
    nx, nv = grid.nx, grid.nv[0]
    hx = grid.L / nx
    hv = (grid.vmax[0] - grid.vmin[0]) / nv
    i0, a = _axis(x, 0.0, hx)
    j0, b = _axis(v, grid.vmin[0], hv)
    da, db = dx / hx, dv / hv
    N, D, fg = (arr.reshape(-1) for arr in reconstruct(grid, x, v.reshape(1, -1), f))
    dN = np.zeros(nx * nv)
    dD = np.zeros(nx * nv)
    for cj in (0, 1):
        wy, dwy = (b, db) if cj else (1.0 - b, -db)
        j = j0 + cj
        inside = (j >= 0) & (j < nv)
        for ci in (0, 1):
            wx, dwx = (a, da) if ci else (1.0 - a, -da)
            col = np.mod(i0 + ci, nx)
            idx = (j * nx + col)[inside]
            w = (wx * wy)[inside]
            dw = (dwx * wy + wx * dwy)[inside]
            np.add.at(dN, idx, dw * f[inside] + w * df[inside])
            np.add.at(dD, idx, dw)
    dfg = np.zeros(nx * nv)
    pos = D > 0.0
    dfg[pos] = (dN[pos] - fg[pos] * dD[pos]) / D[pos]
    return grid.q * hv * dfg.reshape(nv, nx).sum(axis=0)


def field_tangent(grid: Grid, drho):
    """d E of the spectral solve along d rho (the solve is linear)."""
    return poisson(grid.nx, grid.L, grid.cp, np.asarray(drho, dtype=np.float64))[0]
