"""Pins of the oracle's output quantities (Sec. 3.4: field energy, kinetic
energy, the integral of f, the f log f entropy integral, the current density
and the field solver's residual charge) against closed forms.

For a Maxwellian sampled at cell centres the midpoint sum over velocity is
exact up to terms of order exp(-2 pi^2 s^2 / dv^2) (Poisson summation), and
the tails beyond the grid are below 1e-12 here, so the continuum values are
reached to rounding."""
import math

import numpy as np
import pytest

import oracle


def _maxwell_grid(g, n, u, s, amp=0.0, m=1):
    """f on the cell centres of a 1D-1V grid: n (1 + amp cos(k_m x)) M(v; u, s)."""
    dx = g.L / g.nx
    dv = (g.vmax[0] - g.vmin[0]) / g.nv[0]
    x = (np.arange(g.nx) + 0.5) * dx
    v = g.vmin[0] + (np.arange(g.nv[0]) + 0.5) * dv
    M = np.exp(-((v - u) ** 2) / (2 * s * s)) / (s * math.sqrt(2 * math.pi))
    dens = n * (1.0 + amp * np.cos(2 * math.pi * m * x / g.L))
    return np.outer(M, dens), x, v


@pytest.mark.parametrize("u,s,n", [(0.0, 1.0, 1.0), (0.7, 1.3, 0.25), (-1.1, 0.6, 3.0)])
def test_moments_of_a_drifting_maxwellian(u, s, n):
    """N = n L, Ekin = m/2 n L (s^2 + u^2), entropy integral
    n L (log n - log(s sqrt(2 pi)) - 1/2), current density q n u."""
    g = oracle.Grid(1, 64, (320,), 4 * math.pi, (-12.0,), (12.0,), q=-1.0, m=1.7)
    fg, _, _ = _maxwell_grid(g, n, u, s)
    ekin, ntot, ent = oracle.energy(g, fg)
    L = g.L
    assert ntot == pytest.approx(n * L, rel=1e-12)
    assert ekin == pytest.approx(0.5 * g.m * n * L * (s * s + u * u), rel=1e-12)
    assert ent == pytest.approx(n * L * (math.log(n) - math.log(s * math.sqrt(2 * math.pi)) - 0.5), rel=1e-11)
    rho, jx, _ = oracle.moments(g, fg)
    assert np.allclose(rho, g.q * n, rtol=1e-12, atol=0)
    assert np.allclose(jx, g.q * n * u, rtol=1e-11, atol=1e-14)


def test_density_perturbation_averages_out():
    """A cos(k_m x) perturbation sums to zero over the periodic grid, so N and
    Ekin keep their unperturbed values; the current density follows n(x) u."""
    g = oracle.Grid(1, 32, (256,), 5 * math.pi, (-8.0,), (8.0,))
    fg, x, _ = _maxwell_grid(g, 1.0, 0.4, 1.0, amp=0.05, m=3)
    ekin, ntot, _ = oracle.energy(g, fg)
    assert ntot == pytest.approx(g.L, rel=1e-12)
    assert ekin == pytest.approx(0.5 * g.L * (1.0 + 0.16), rel=1e-12)
    _, jx, _ = oracle.moments(g, fg)
    want = g.q * 0.4 * (1.0 + 0.05 * np.cos(2 * math.pi * 3 * x / g.L))
    assert np.max(np.abs(jx - want)) <= 1e-12


def test_1d3v_isotropic_maxwellian():
    """Three velocity dimensions: Ekin = m/2 n L (3 s^2 + u_x^2), N = n L."""
    nv = 30
    g = oracle.Grid(3, 16, (nv, nv, nv), 2 * math.pi, (-9.0, -9.0, -9.0), (9.0, 9.0, 9.0))
    dv = 18.0 / nv
    v = -9.0 + (np.arange(nv) + 0.5) * dv
    u, s, n = 0.8, 1.0, 0.5
    Mx = np.exp(-((v - u) ** 2) / (2 * s * s)) / (s * math.sqrt(2 * math.pi))
    My = np.exp(-(v ** 2) / (2 * s * s)) / (s * math.sqrt(2 * math.pi))
    f3 = n * My[:, None, None] * My[None, :, None] * Mx[None, None, :]      # (vz, vy, vx)
    fg = np.repeat(f3[..., None], g.nx, axis=3)
    ekin, ntot, ent = oracle.energy(g, fg)
    assert ntot == pytest.approx(n * g.L, rel=1e-11)
    assert ekin == pytest.approx(0.5 * n * g.L * (3 * s * s + u * u), rel=1e-11)
    want_S = n * g.L * (math.log(n) - 3 * math.log(s * math.sqrt(2 * math.pi)) - 1.5)
    assert ent == pytest.approx(want_S, rel=1e-10)


@pytest.mark.parametrize("nx", [16, 64, 512])
def test_field_energy_of_one_mode(nx):
    """E = A sin(k_m x): sum over whole periods of sin^2 is nx/2, so
    W = A^2 L / (4 c_p)."""
    L, cp, A = 3.0, 4 * math.pi, 0.3
    x = (np.arange(nx) + 0.5) * L / nx
    for m in (1, 3, nx // 2 - 1):
        E = A * np.sin(2 * math.pi * m * x / L)
        assert oracle.field_energy(nx, L, cp, E) == pytest.approx(A * A * L / (4 * cp), rel=1e-12)


@pytest.mark.parametrize("nx", [16, 128, 1024])
def test_residual_charge_closed_form(nx):
    """The solve gives E_hat = -i c_p kappa / K^2 rho_hat with kappa = sin(k dx)/dx
    and K^2 = (2 sin(k dx/2)/dx)^2; a centred difference multiplies E_hat by
    i sin(k dx)/dx, so it returns c_p cos^2(k dx/2) rho_hat and the residual of
    a single mode rho = A cos(k x) + c is A sin^2(k dx/2) cos(k x) (the constant
    c is the neutralising background).  At the Nyquist mode the field is zero
    and the residual is the whole mode, which the same formula gives."""
    L, cp, A, c = 7.0, 1.0, 0.8, -1.3
    dx = L / nx
    x = (np.arange(nx) + 0.5) * dx
    for m in (1, 5, nx // 4, nx // 2 - 1, nx // 2):
        k = 2 * math.pi * m / L
        rho = A * np.cos(k * x) + c
        E, _ = oracle.poisson(nx, L, cp, rho)
        got = oracle.residual(nx, L, cp, rho, E)
        want = A * math.sin(0.5 * k * dx) ** 2 * np.cos(k * x)
        assert np.max(np.abs(got - want)) <= 1e-12 * A, m

