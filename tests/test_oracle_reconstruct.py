"""Pins of the oracle's reconstruction (Eq. (reconstruction), Sec. 2) against
things other than itself: a hand-derived fixture, the literal area-overlap
picture in exact arithmetic, closed forms and invariants."""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from physics import cic_overlap_bruteforce

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _frac(s):
    return float(Fraction(s))


def test_hand_derived_2x2():
    grid_line, markers, cells = None, [], []
    for line in open(os.path.join(GOLDEN, "reconstruct_2x2_hand.txt")):
        if line.startswith("#") or not line.strip():
            continue
        tok = line.split()
        if tok[0] == "grid":
            grid_line = tok[1:]
        elif tok[0] == "marker":
            markers.append([float(t) for t in tok[1:]])
        elif tok[0] == "cell":
            cells.append((int(tok[1]), int(tok[2]), _frac(tok[3]), _frac(tok[4]), _frac(tok[5])))
    nx, L, nv, vmin, vmax = int(grid_line[0]), float(grid_line[1]), int(grid_line[2]), float(grid_line[3]), float(grid_line[4])
    g = oracle.Grid(1, nx, (nv,), L, (vmin,), (vmax,))
    m = np.array(markers)
    N, D, f = oracle.reconstruct(g, m[:, 0], m[:, 1], m[:, 2])
    for i, j, n_, d_, f_ in cells:
        assert N[j, i] == pytest.approx(n_, rel=1e-15, abs=0)
        assert D[j, i] == pytest.approx(d_, rel=1e-15, abs=0)
        assert f[j, i] == pytest.approx(f_, rel=1e-15, abs=0)


def _dyadic_markers(rng, n, nx, L, nv, vmin, vmax, bits=6):
    """Markers on a dyadic lattice so every weight is exact in binary floating point."""
    xs = rng.integers(0, nx * 2 ** bits, n) * (L / (nx * 2 ** bits))
    vs = vmin + rng.integers(-2 ** bits, (nv + 1) * 2 ** bits, n) * ((vmax - vmin) / (nv * 2 ** bits))
    fs = rng.integers(1, 64, n) / 16.0
    return xs, vs, fs


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("nx,nv", [(2, 2), (4, 4), (4, 3)])
def test_area_overlap_bruteforce_1d1v(seed, nx, nv):
    """Against the literal overlap area, including x wrap and clouds that stick
    out of the velocity range (below vmin and above vmax)."""
    rng = np.random.default_rng(seed)
    L, vmin, vmax = 4.0, -2.0, 2.0
    xs, vs, fs = _dyadic_markers(rng, 3 + seed, nx, L, nv, vmin, vmax)
    g = oracle.Grid(1, nx, (nv,), L, (vmin,), (vmax,))
    N, D, f = oracle.reconstruct(g, xs, vs, fs)
    Nb, Db = cic_overlap_bruteforce(nx, L, (nv,), (vmin,), (vmax,),
                                    [(x, (v,), ff) for x, v, ff in zip(xs, vs, fs)])
    for j in range(nv):
        for i in range(nx):
            assert D[j, i] == pytest.approx(float(Db.get((i, j), 0)), abs=1e-15)
            assert N[j, i] == pytest.approx(float(Nb.get((i, j), 0)), abs=1e-15)
            dd = Db.get((i, j), 0)
            want = float(Nb[(i, j)] / dd) if dd else 0.0
            assert f[j, i] == pytest.approx(want, rel=1e-15, abs=0)


def test_area_overlap_bruteforce_1d3v():
    rng = np.random.default_rng(7)
    nx, nvs, L = 2, (2, 3, 2), 2.0
    vmin, vmax = (-1.0, -1.5, 0.0), (1.0, 1.5, 2.0)
    ms = []
    for _ in range(4):
        x = rng.integers(0, nx * 8) * (L / (nx * 8))
        v = tuple(vmin[d] + rng.integers(-4, (nvs[d] + 1) * 8) * ((vmax[d] - vmin[d]) / (nvs[d] * 8)) for d in range(3))
        ms.append((x, v, rng.integers(1, 16) / 8.0))
    g = oracle.Grid(3, nx, nvs, L, vmin, vmax)
    N, D, f = oracle.reconstruct(g, np.array([m[0] for m in ms]),
                                 np.array([[m[1][d] for m in ms] for d in range(3)]),
                                 np.array([m[2] for m in ms]))
    Nb, Db = cic_overlap_bruteforce(nx, L, nvs, vmin, vmax, ms)
    for jz in range(nvs[2]):
        for jy in range(nvs[1]):
            for jx in range(nvs[0]):
                for i in range(nx):
                    key = (i, jx, jy, jz)
                    assert D[jz, jy, jx, i] == pytest.approx(float(Db.get(key, 0)), abs=1e-15)
                    assert N[jz, jy, jx, i] == pytest.approx(float(Nb.get(key, 0)), abs=1e-15)


def test_constant_f_is_reproduced_exactly():
    """f_l = c (a power of two) gives N = c D bit for bit, so f_g = c wherever D > 0."""
    rng = np.random.default_rng(3)
    nx, nv, L, vmin, vmax = 16, 12, 5.0, -3.0, 3.0
    n = 4000
    x = rng.uniform(0, L, n)
    v = rng.uniform(vmin - 0.3, vmax + 0.3, n)
    c = 0.25
    g = oracle.Grid(1, nx, (nv,), L, (vmin,), (vmax,))
    N, D, f = oracle.reconstruct(g, x, v, np.full(n, c))
    assert np.all(f[D > 0] == c)
    assert np.all(N == c * D)


def test_cell_centred_markers_are_identity():
    """One marker at each cell centre: every cloud coincides with its cell."""
    nx, nv = 8, 8
    L, vmin, vmax = 8.0, -4.0, 4.0   # dx = dv = 1: centres are exact
    i, j = np.meshgrid(np.arange(nx), np.arange(nv))
    x = (i.ravel() + 0.5) * 1.0
    v = vmin + (j.ravel() + 0.5) * 1.0
    fl = np.arange(nx * nv, dtype=float) + 1.0
    g = oracle.Grid(1, nx, (nv,), L, (vmin,), (vmax,))
    N, D, f = oracle.reconstruct(g, x, v, fl)
    assert np.array_equal(D, np.ones((nv, nx)))
    assert np.array_equal(f.ravel(), fl)


def test_conservation_of_weight_and_mass():
    """Sum_g D_g counts every marker whose cloud is inside the velocity range
    once; Sum_g N_g is the sum of their f (Eq. (reconstruction) weights sum to 1)."""
    rng = np.random.default_rng(11)
    nx, nv, L, vmin, vmax = 32, 20, 7.0, -5.0, 5.0
    dv = (vmax - vmin) / nv
    n = 20000
    x = rng.uniform(0, L, n)
    v = rng.uniform(vmin + dv / 2, vmax - dv / 2, n)   # clouds fully inside
    fl = rng.uniform(0.1, 2.0, n)
    g = oracle.Grid(1, nx, (nv,), L, (vmin,), (vmax,))
    N, D, f = oracle.reconstruct(g, x, v, fl)
    assert D.sum() == pytest.approx(n, rel=1e-13)
    assert N.sum() == pytest.approx(fl.sum(), rel=1e-13)


def test_vhs_does_not_drown_low_weight_markers():
    """Two markers share one cell with f = 1 and 1e-8: the normalised VHS
    reconstruction gives their weighted mean (about 0.5) where the naive PIC
    deposit gives about 1 (Sec. 2, the comparison of the two sums)."""
    g = oracle.Grid(1, 4, (4,), 4.0, (0.0,), (4.0,))
    x = np.array([1.5, 1.5])
    v = np.array([1.5, 1.5])
    fl = np.array([1.0, 1e-8])
    N, D, f = oracle.reconstruct(g, x, v, fl)
    naive = oracle.deposit_naive(g, x, v, fl)
    assert f[1, 1] == pytest.approx((1.0 + 1e-8) / 2, rel=1e-15)
    assert naive[1, 1] == pytest.approx(1.0 + 1e-8, rel=1e-15)


def test_permutation_changes_only_rounding():
    rng = np.random.default_rng(5)
    nx, nv, L, vmin, vmax = 32, 32, 6.0, -6.0, 6.0
    n = 30000
    x = rng.uniform(0, L, n)
    v = rng.normal(0, 2, n)
    fl = np.exp(rng.uniform(-18, 0, n))
    g = oracle.Grid(1, nx, (nv,), L, (vmin,), (vmax,))
    N1, D1, f1 = oracle.reconstruct(g, x, v, fl)
    p = rng.permutation(n)
    N2, D2, f2 = oracle.reconstruct(g, x[p], v[p], fl[p])
    assert np.max(np.abs(N1 - N2)) <= 1e-14 * np.max(np.abs(N1))
    assert np.max(np.abs(f1 - f2)) <= 1e-14 * np.max(np.abs(f1))


def test_1d3v_reduces_to_1d1v():
    """Replicating a 1D-1V population at every (vy, vz) cell centre gives the
    1D-1V reconstruction in every (vy, vz) plane, and the same rho."""
    rng = np.random.default_rng(9)
    nx, nvx, nvy, nvz = 8, 6, 3, 2
    L = 4.0
    g1 = oracle.Grid(1, nx, (nvx,), L, (-3.0,), (3.0,))
    g3 = oracle.Grid(3, nx, (nvx, nvy, nvz), L, (-3.0, -1.5, -1.0), (3.0, 1.5, 1.0))
    n = 500
    x = rng.uniform(0, L, n)
    vx = rng.uniform(-2.5, 2.5, n)
    fl = rng.uniform(0.5, 1.5, n)
    N1, D1, f1 = oracle.reconstruct(g1, x, vx, fl)
    vy_c = -1.5 + (np.arange(nvy) + 0.5) * 1.0
    vz_c = -1.0 + (np.arange(nvz) + 0.5) * 1.0
    X, VX, VY, VZ, F = [], [], [], [], []
    for a in vy_c:
        for b in vz_c:
            X.append(x); VX.append(vx); VY.append(np.full(n, a)); VZ.append(np.full(n, b)); F.append(fl / (nvy * nvz))
    x3, vx3, vy3, vz3, f3 = map(np.concatenate, (X, VX, VY, VZ, F))
    N3, D3, fg3 = oracle.reconstruct(g3, x3, np.stack([vx3, vy3, vz3]), f3)
    for jz in range(nvz):
        for jy in range(nvy):
            np.testing.assert_allclose(fg3[jz, jy] * nvy * nvz, f1, rtol=1e-14, atol=0)
    rho1, _, _ = oracle.moments(g1, f1)
    rho3, _, _ = oracle.moments(g3, fg3)
    np.testing.assert_allclose(rho3, rho1, rtol=1e-14)
