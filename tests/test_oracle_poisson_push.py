"""Pins of the oracle's field solve (Eq. (poissonk), Eq. (kappasoftening)),
moments, gather and push against closed forms and an independent real-space
finite-difference solve."""
import math

import numpy as np
import pytest

import oracle


@pytest.mark.parametrize("nx", [8, 64, 1024])
@pytest.mark.parametrize("m", [1, 3])
def test_single_mode_closed_form(nx, m):
    """rho = A cos(k x_i) gives E_i = cp A kappa/K^2 sin(k x_i)."""
    L, cp, A = 20.0 * math.pi, 1.0, 0.37
    dx = L / nx
    xi = (np.arange(nx) + 0.5) * dx
    k = 2 * math.pi * m / L
    rho = A * np.cos(k * xi)
    E, m1 = oracle.poisson(nx, L, cp, rho)
    kappa = math.sin(k * dx) / dx
    K2 = (2.0 * math.sin(0.5 * k * dx) / dx) ** 2
    want = cp * A * kappa / K2 * np.sin(k * xi)
    assert np.max(np.abs(E - want)) <= 1e-13 * np.max(np.abs(want))
    if m == 1:
        assert m1 == pytest.approx(cp * A * kappa / K2, rel=1e-12)


def _fd_solve(rho, dx, cp):
    """Real-space solve: the sinc-softened operators are exactly the centred
    first difference (kappa) and the three-point Laplacian (K^2), so E is
    -(phi_{i+1} - phi_{i-1})/(2 dx) with (phi_{i+1} - 2 phi_i + phi_{i-1})/dx^2
    = -cp (rho_i - mean rho), phi periodic.  Solved by two cumulative sums."""
    nx = rho.size
    r = rho - rho.mean()
    # second difference of phi: d2[i] = -cp r[i] dx^2; first differences g[i] = phi[i+1]-phi[i]
    d2 = -cp * r * dx * dx
    g = np.concatenate([[0.0], np.cumsum(d2[1:])])  # g[i] - g[i-1] = d2[i], periodic up to a constant
    g -= g.mean()                                      # sum of first differences of a periodic phi is 0
    phi = np.concatenate([[0.0], np.cumsum(g[:-1])])
    return -(np.roll(phi, -1) - np.roll(phi, 1)) / (2 * dx)


@pytest.mark.parametrize("nx", [16, 128, 512])
def test_equals_real_space_finite_differences(nx):
    rng = np.random.default_rng(nx)
    L, cp = 5.0 * math.pi, 4.0 * math.pi
    rho = rng.normal(size=nx)
    # drop the Nyquist component, which the spectral solve zeroes by choice
    rhat = np.fft.fft(rho)
    rhat[nx // 2] = 0.0
    rho = np.fft.ifft(rhat).real
    E, _ = oracle.poisson(nx, L, cp, rho)
    Efd = _fd_solve(rho, L / nx, cp)
    assert np.max(np.abs(E - Efd)) <= 1e-12 * np.max(np.abs(Efd))


def test_invariants():
    nx, L, cp = 64, 4 * math.pi, 1.0
    rng = np.random.default_rng(1)
    a, b = rng.normal(size=nx), rng.normal(size=nx)
    Ea, _ = oracle.poisson(nx, L, cp, a)
    Eb, _ = oracle.poisson(nx, L, cp, b)
    Eab, _ = oracle.poisson(nx, L, cp, 2.0 * a - 3.0 * b)
    s = np.max(np.abs(Eab))
    assert abs(Ea.sum()) <= 1e-13 * np.abs(Ea).sum()                      # E_hat_0 = 0
    assert np.max(np.abs(Eab - (2 * Ea - 3 * Eb))) <= 1e-13 * s            # linearity
    Ec, _ = oracle.poisson(nx, L, cp, np.full(nx, 3.5))
    assert np.max(np.abs(Ec)) <= 1e-14                                     # neutralising background
    alt = np.array([(-1.0) ** i for i in range(nx)])
    En, _ = oracle.poisson(nx, L, cp, alt)                                # pure Nyquist input
    assert np.max(np.abs(En)) <= 1e-14
    E4, _ = oracle.poisson(nx, L, 4 * math.pi, a)                          # CGS constant scales E
    assert np.max(np.abs(E4 - 4 * math.pi * Ea)) <= 1e-13 * np.max(np.abs(E4))


def test_moments_midpoint_rule_on_maxwellian():
    """rho from cell-centred samples of a unit Maxwellian is the midpoint rule:
    dv sum M(v_j) = 1 up to the tails beyond +-6 and the O(dv^2) midpoint error."""
    nx, nv = 4, 240
    g = oracle.Grid(1, nx, (nv,), 1.0, (-6.0,), (6.0,), q=-1.0)
    vj = -6.0 + (np.arange(nv) + 0.5) * (12.0 / nv)
    M = np.exp(-vj ** 2 / 2) / math.sqrt(2 * math.pi)
    fg = np.repeat(M[:, None], nx, axis=1)
    rho, jx, m2 = oracle.moments(g, fg)
    tail = math.erfc(6.0 / math.sqrt(2.0))
    assert rho == pytest.approx(np.full(nx, -(1.0 - tail)), abs=1e-8)
    assert jx == pytest.approx(np.zeros(nx), abs=1e-13)
    assert m2 == pytest.approx(np.ones(nx), abs=1e-6)


def test_gather_is_area_weighting():
    """A marker at a cell centre sees E_i; halfway between centres the mean;
    near x = 0 and x = L the periodic neighbour (Sec. 2: the field goes back to
    the markers with the same area weighting as the reconstruction)."""
    nx, L = 8, 8.0
    g = oracle.Grid(1, nx, (4,), L, (-1.0,), (1.0,), dt=1.0, q=1.0, m=1.0)
    E = np.arange(nx, dtype=float) * 0.5 + 1.0
    x = np.array([2.5, 3.0, 0.25, 7.75, 7.5])
    v0 = np.zeros(5)
    # with dt = 1 and q/m = 1 the velocity after one kick is the gathered field
    _, v1 = oracle.push(g, x, v0, E, kick=1.0)
    want = [E[2], 0.5 * (E[2] + E[3]), 0.25 * E[0] + 0.75 * E[7] + 0.0, 0.75 * E[7] + 0.25 * E[0], E[7]]
    want[2] = 0.75 * E[0] + 0.25 * E[7]
    np.testing.assert_allclose(v1[0], want, rtol=1e-15)


def test_free_streaming_and_uniform_force():
    nx, L, dt = 16, 10.0, 0.1
    rng = np.random.default_rng(2)
    x0 = rng.uniform(0, L, 1000)
    v0 = rng.normal(size=1000)
    g0 = oracle.Grid(1, nx, (8,), L, (-4.0,), (4.0,), dt=dt, q=0.0, m=1.0)
    x, v = x0, v0[None]
    for _ in range(50):
        x, v = oracle.push(g0, x, v, np.zeros(nx))
    want = np.mod(x0 + 50 * v0 * dt, L)
    d = np.abs(x - want)
    d = np.minimum(d, L - d)
    assert d.max() <= 1e-12 and np.all((x >= 0) & (x < L))
    g1 = oracle.Grid(1, nx, (8,), L, (-4.0,), (4.0,), dt=dt, q=-2.0, m=4.0)
    E = np.full(nx, 0.3)
    x, v = x0, v0[None]
    for _ in range(40):
        x, v = oracle.push(g1, x, v, E)
    np.testing.assert_allclose(v[0], v0 + 40 * (-0.5) * 0.3 * dt, atol=1e-13)


def test_wrap_stays_in_domain():
    g = oracle.Grid(1, 4, (2,), 1.0, (-1.0,), (1.0,), dt=1.0, q=0.0)
    x = np.array([0.0, 0.999999, 1e-17, 0.5])
    v = np.array([[-1e-17, 1e-6, -1e-17, -0.5]])
    xn, _ = oracle.push(g, x, v, np.zeros(4))
    assert np.all((xn >= 0.0) & (xn < 1.0))


def _grid3(B, dt=0.3, q=-1.0, m=1.0):
    return oracle.Grid(3, 8, (4, 4, 4), 2 * math.pi, (-6.0,) * 3, (6.0,) * 3, dt=dt, q=q, m=m, B=B)


def test_boris_speed_and_rotation_angle():
    """With E = 0 the magnetised push keeps |v| and v.b, and turns the
    perpendicular velocity about b = B/|B| by -2 atan((q/m)|B| dt/2) per step
    (the Boris angle); for a short step the change of v points along
    (q/m) v x B, the sense of the Lorentz force."""
    Bv = np.array([0.0, 3.0, 4.0]) / 5.0 * 0.7
    g = _grid3(tuple(Bv))
    rng = np.random.default_rng(3)
    n = 5
    x0 = rng.uniform(0, g.L, n)
    v0 = rng.normal(size=(3, n))
    b = Bv / np.linalg.norm(Bv)
    theta = -2.0 * math.atan(0.5 * (g.q / g.m) * np.linalg.norm(Bv) * g.dt)
    xs, vs = x0, v0
    E = np.zeros(g.nx)
    for step in range(1, 8):
        xs, vs = oracle.push(g, xs, vs, E)
        assert np.allclose(np.linalg.norm(vs, axis=0), np.linalg.norm(v0, axis=0), rtol=1e-14, atol=0)
        assert np.allclose(b @ vs, b @ v0, rtol=0, atol=1e-14)
        p0 = v0 - np.outer(b, b @ v0)
        p1 = vs - np.outer(b, b @ vs)
        ang = np.arctan2(b @ np.cross(p0.T, p1.T).T, np.sum(p0 * p1, axis=0))
        want = math.remainder(step * theta, 2 * math.pi)
        assert np.allclose(ang, want, rtol=0, atol=1e-12)
    g2 = _grid3(tuple(Bv), dt=1e-6)
    _, v1 = oracle.push(g2, x0, v0, E)
    lorentz = (g.q / g.m) * np.cross(v0.T, Bv).T * g2.dt
    assert np.allclose(v1 - v0, lorentz, rtol=1e-5, atol=1e-16)


def test_boris_e_cross_b_drift_is_a_fixed_point():
    """Uniform E along x and B along z: the E x B drift velocity
    v_d = E x B / |B|^2 = -(E/B) y_hat is reproduced exactly (a fixed point of
    the scheme), and a gyrating marker's mean y velocity over whole turns is
    v_d (checked over 400 steps, about 30 turns)."""
    E0, B0 = 0.2, 0.8
    g = _grid3((0.0, 0.0, B0), dt=0.25)
    E = np.full(g.nx, E0)
    x = np.array([1.0])
    v = np.array([[0.0], [-E0 / B0], [0.3]])
    xs, vs = x, v
    for _ in range(50):
        xs, vs = oracle.push(g, xs, vs, E)
    assert np.allclose(vs, v, rtol=0, atol=1e-14)
    assert abs(xs[0] - x[0]) <= 1e-14
    vg = np.array([[0.9], [-E0 / B0 + 0.4], [0.0]])
    theta = 2.0 * math.atan(0.5 * abs(g.q / g.m) * B0 * g.dt)
    nturn = int(round(30 * 2 * math.pi / theta))
    acc = 0.0
    xs, vs = x, vg
    for _ in range(nturn):
        xs, vs = oracle.push(g, xs, vs, E)
        acc += vs[1, 0]
    assert abs(acc / nturn - (-E0 / B0)) <= 0.01 * E0 / B0


def test_boris_without_field_is_the_plain_kick():
    """B = 0 in 1D-3V leaves vy, vz untouched and kicks vx exactly as the
    unmagnetised push."""
    g = _grid3((0.0, 0.0, 0.0))
    rng = np.random.default_rng(5)
    x = rng.uniform(0, g.L, 6)
    v = rng.normal(size=(3, 6))
    E = rng.normal(size=g.nx)
    xs, vs = oracle.push(g, x, v, E)
    dx = g.L / g.nx
    s = x / dx - 0.5
    i0 = np.floor(s).astype(int)
    a = s - i0
    El = (1 - a) * E[i0 % g.nx] + a * E[(i0 + 1) % g.nx]
    assert np.array_equal(vs[1:], v[1:])
    assert np.allclose(vs[0], v[0] + (g.q / g.m) * El * g.dt, rtol=0, atol=1e-15)


@pytest.mark.parametrize("nx", [64, 1024, 4096])
def test_constant_offset_leaves_field_unchanged(nx):
    """E_hat_0 = 0 (Eq. (poissonk)): adding a constant to rho cannot change E.
    The constant here is the size of the neutralised charge and far larger than
    the fluctuation, as in every plasma run (rho ~ -1 + 1e-4 modes); the offset
    values are chosen on a 2^-52 grid so that 1 + r is exact in FP64.  A solve
    that lets the mean leak into the other modes through rounded twiddles
    misses this by ~1e-11 of max|E|."""
    rng = np.random.default_rng(nx + 7)
    L, cp = 20.0 * math.pi, 1.0
    xi = (np.arange(nx) + 0.5) * (L / nx)
    r = sum(1e-4 * np.cos(0.1 * m * xi + rng.uniform(0, 2 * math.pi)) for m in range(1, 17))
    r = np.round(r * 2.0 ** 52) * 2.0 ** -52
    E_small, _ = oracle.poisson(nx, L, cp, r)
    for dc in (-1.0, 1.0, 1.5):
        big = dc + r
        assert np.array_equal(big - dc, r)            # the offset is exact
        E_big, _ = oracle.poisson(nx, L, cp, big)
        assert np.max(np.abs(E_big - E_small)) <= 1e-14 * np.max(np.abs(E_small))
    # and the offset-free solve itself is the finite-difference one
    rhat = np.fft.fft(r)
    rhat[nx // 2] = 0.0
    rr = np.fft.ifft(rhat).real
    E_rr, _ = oracle.poisson(nx, L, cp, rr)
    assert np.max(np.abs(E_rr - _fd_solve(rr, L / nx, cp))) <= 1e-12 * np.max(np.abs(E_rr))
