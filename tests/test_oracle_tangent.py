"""Pins of the oracle's tangent-linear stage maps (oracle/tangent.py) against
the oracle's own forward stages, by central differences and exact cases.

The push is linear inside a cell and the field solve linear everywhere, so
their differences agree with the tangents to rounding.  Reconstruction and
moments are linear in the weights f (differences exact to rounding) and
rational in the positions (second-order central differences, step 1e-6 of a
cell, agree to ~1e-7 relative).  Markers are kept 5% of a cell away from the
cell-centre lines so that no step crosses one.  A uniform f reconstructs to
the same uniform value in every touched cell, so moving markers inside their
cells leaves rho unchanged: the position tangent of that state is zero.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import tangent


def _grid(nx=16, nv=12, q=-1.0, cp=1.0):
    return oracle.Grid(1, nx, (nv,), 4 * math.pi, (-5.0,), (5.0,), dt=0.1, q=q, m=1.0, cp=cp)


def _markers(g, n, rng, margin=0.05):
    hx = g.L / g.nx
    hv = (g.vmax[0] - g.vmin[0]) / g.nv[0]
    # offsets past the lower cell centre kept inside [margin, 1 - margin]
    ix = rng.integers(0, g.nx, n)
    jv = rng.integers(-1, g.nv[0], n)            # -1 and nv-1: a corner outside the grid
    a = rng.uniform(margin, 1 - margin, n)
    b = rng.uniform(margin, 1 - margin, n)
    x = (ix + 0.5 + a) * hx
    x = np.where(x >= g.L, x - g.L, x)
    v = g.vmin[0] + (jv + 0.5 + b) * hv
    f = rng.uniform(0.1, 2.0, n)
    return x, v, f


def _rho(g, x, v, f):
    _, _, fg = oracle.reconstruct(g, x, v.reshape(1, -1), f)
    return oracle.moments(g, fg)[0]


def test_push_tangent_matches_differences():
    g = _grid()
    rng = np.random.default_rng(1)
    x, v, _ = _markers(g, 300, rng)
    E = rng.normal(size=g.nx)
    dx, dv, dE = rng.normal(size=x.size), rng.normal(size=x.size), rng.normal(size=g.nx)
    hx = g.L / g.nx
    for kick in (1.0, 0.5):
        tx, tv = tangent.push_tangent(g, x, v, E, kick, dx, dv, dE)
        h = 1e-6 * hx / np.max(np.abs(dx))
        xp, vp = oracle.push(g, x + h * dx, v + h * dv, E + h * dE, kick)
        xm, vm = oracle.push(g, x - h * dx, v - h * dv, E - h * dE, kick)
        # undo the periodic wrap before differencing
        ddx = np.mod(xp - xm + 0.5 * g.L, g.L) - 0.5 * g.L
        fx = ddx / (2 * h)
        fv = (vp - vm)[0] / (2 * h)
        assert np.max(np.abs(fx - tx)) <= 1e-7 * np.max(np.abs(tx))
        assert np.max(np.abs(fv - tv)) <= 1e-7 * np.max(np.abs(tv))


def test_push_tangent_of_field_only_is_the_interpolation():
    """Along dE alone: dv' = c sum_i W_i(x) dE_i and dx' = dt dv', W the
    cloud-in-cell weights of the marker's two neighbouring cells."""
    g = _grid(nx=8)
    x = np.array([0.75 * g.L / g.nx + 0.0, 3.2 * g.L / g.nx])      # a = 0.25 and 0.7 past centres 0 and 2
    v = np.zeros(2)
    E = np.zeros(g.nx)
    dE = np.arange(1.0, g.nx + 1.0)
    tx, tv = tangent.push_tangent(g, x, v, E, 1.0, np.zeros(2), np.zeros(2), dE)
    c = g.q / g.m * g.dt
    want = c * np.array([0.75 * 1.0 + 0.25 * 2.0, 0.3 * 3.0 + 0.7 * 4.0])
    assert np.allclose(tv, want, rtol=1e-14, atol=0)
    assert np.allclose(tx, g.dt * want, rtol=1e-14, atol=0)


def test_deposit_tangent_in_the_weights_is_exact():
    g = _grid()
    rng = np.random.default_rng(2)
    x, v, f = _markers(g, 500, rng)
    df = rng.normal(size=f.size)
    z = np.zeros_like(x)
    t = tangent.deposit_tangent(g, x, v, f, z, z, df)
    fd = (_rho(g, x, v, f + df) - _rho(g, x, v, f - df)) / 2.0
    assert np.max(np.abs(fd - t)) <= 1e-13 * np.max(np.abs(t))


def test_deposit_tangent_in_the_positions_matches_differences():
    g = _grid()
    rng = np.random.default_rng(3)
    x, v, f = _markers(g, 500, rng)
    dx, dv = rng.normal(size=x.size), rng.normal(size=x.size)
    df = rng.normal(size=x.size)
    t = tangent.deposit_tangent(g, x, v, f, dx, dv, df)
    hx = g.L / g.nx
    h = 1e-6 * hx / max(np.max(np.abs(dx)), np.max(np.abs(dv)))
    fd = (_rho(g, x + h * dx, v + h * dv, f + h * df) - _rho(g, x - h * dx, v - h * dv, f - h * df)) / (2 * h)
    assert np.max(np.abs(fd - t)) <= 1e-6 * np.max(np.abs(t))


def test_deposit_tangent_of_uniform_weights_vanishes():
    g = _grid()
    rng = np.random.default_rng(4)
    x, v, _ = _markers(g, 400, rng)
    f = np.full(x.size, 1.5)
    t = tangent.deposit_tangent(g, x, v, f, rng.normal(size=x.size), rng.normal(size=x.size), np.zeros(x.size))
    assert np.max(np.abs(t)) <= 1e-13


def test_field_tangent_is_the_solve():
    g = _grid(nx=32, cp=4 * math.pi)
    rng = np.random.default_rng(5)
    r1, r2 = rng.normal(size=g.nx), rng.normal(size=g.nx)
    a, b = 0.3, -1.7
    lhs = tangent.field_tangent(g, a * r1 + b * r2)
    rhs = a * tangent.field_tangent(g, r1) + b * tangent.field_tangent(g, r2)
    assert np.max(np.abs(lhs - rhs)) <= 1e-13 * np.max(np.abs(lhs))


@pytest.mark.parametrize("nx", [8, 32, 128])
def test_field_solve_is_antisymmetric(nx):
    """<P r, m> = -<r, P m>: the transfer function -i c_p kappa/K^2 is odd and
    imaginary, the mean and the Nyquist mode are removed on both sides."""
    g = _grid(nx=nx)
    rng = np.random.default_rng(nx)
    r, m = rng.normal(size=nx), rng.normal(size=nx)
    lhs = float(np.dot(tangent.field_tangent(g, r), m))
    rhs = -float(np.dot(r, tangent.field_tangent(g, m)))
    scale = float(np.sum(np.abs(tangent.field_tangent(g, r) * m)))
    assert abs(lhs - rhs) <= 1e-13 * scale
