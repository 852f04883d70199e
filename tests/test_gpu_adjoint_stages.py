"""Dot-product checks of the library's reverse stages, one stage at a time.

For each stage S of the 1D-1V step (Sec. 2) with tangent map J (the oracle's
oracle/tangent.py, pinned by the CPU tests against differences of the oracle's
forward stages) and the library's reverse stage R (avl_adjoint_push,
avl_adjoint_deposit, avl_adjoint_field), the identity <J du, lam> = <du, R lam>
is checked for random directions du and adjoints lam at 1e-12 of the sum of
the magnitudes of the terms (FP64; 1e-5 for the FP32 storage form, whose f and
D grids are FP32).

States are random markers at 8 per cell on a 32 x 24 grid, velocities kept a
cell inside the grid, so that every touched cell has D of order one and both
sides see the same cell for every marker.  The integer-summed field adjoint
of the push is also checked to be bit-identical under a permutation of the
markers.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from oracle import tangent
from paper_1804_03901_amd import avl, inputs

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _case(precision, seed=7, nx=32, nv=24, ppc=8):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    w = inputs.bump_on_tail(nx=nx, nv=nv, ppc=ppc, seed=seed)
    rng = np.random.default_rng(seed)
    n = nx * nv * ppc
    hv = (w.vmax[0] - w.vmin[0]) / nv
    x = rng.uniform(0.0, w.L, n)
    v = rng.uniform(w.vmin[0] + hv, w.vmax[0] - hv, n)
    f = rng.uniform(0.2, 2.0, n)
    print(f"[case] {w.name} prec={precision} n={n}", flush=True)
    sim = avl.Simulation(w, x, v, f, precision=precision)
    return w, sim, oracle.Grid.from_workload(w), rng


def _t(a):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda:0")


def _check(lhs_terms, rhs_terms, tol, what):
    lhs = sum(float(np.sum(t)) for t in lhs_terms)
    rhs = sum(float(np.sum(t)) for t in rhs_terms)
    scale = sum(float(np.sum(np.abs(t))) for t in lhs_terms + rhs_terms)
    print(f"[result] {what}: <J du, lam> = {lhs:.15e}, <du, R lam> = {rhs:.15e}, rel {abs(lhs - rhs) / scale:.2e}",
          flush=True)
    assert abs(lhs - rhs) <= tol * scale, (what, lhs, rhs, scale)


@pytest.mark.parametrize("kick", [1.0, 0.5])
def test_push_stage_dot_product(kick):
    w, sim, g, rng = _case(avl.AVL_FP64)
    n = sim.n
    x = rng.uniform(0.0, w.L, n)
    v = rng.normal(size=n)
    E = rng.normal(size=w.nx)
    lx1, lv1 = rng.normal(size=n), rng.normal(size=n)
    lx, lv, Eb = (torch.empty(k, dtype=torch.float64, device="cuda:0") for k in (n, n, w.nx))
    avl.avl_adjoint_push(sim.h, _t(x), _t(E), kick, _t(lx1), _t(lv1), lx, lv, Eb)
    torch.cuda.synchronize()
    lx, lv, Eb = lx.cpu().numpy(), lv.cpu().numpy(), Eb.cpu().numpy()
    for trial in range(3):
        dx, dv, dE = rng.normal(size=n), rng.normal(size=n), rng.normal(size=w.nx)
        tx, tv = tangent.push_tangent(g, x, v, E, kick, dx, dv, dE)
        _check([tx * lx1, tv * lv1], [dx * lx, dv * lv, dE * Eb], TOL, f"push kick={kick} #{trial}")
    sim.check()


def test_push_stage_in_place_and_order_free():
    """In place (lam_x == lam_x_in) gives the same adjoints, and the field
    adjoint of permuted markers is the same bit for bit."""
    w, sim, g, rng = _case(avl.AVL_FP64)
    n = sim.n
    x = rng.uniform(0.0, w.L, n)
    E = rng.normal(size=w.nx)
    lx1, lv1 = rng.normal(size=n) * 1e3, rng.normal(size=n)
    out = [torch.empty(k, dtype=torch.float64, device="cuda:0") for k in (n, n, w.nx)]
    avl.avl_adjoint_push(sim.h, _t(x), _t(E), 1.0, _t(lx1), _t(lv1), *out)
    ax, av = _t(lx1), _t(lv1)
    Eb2 = torch.empty(w.nx, dtype=torch.float64, device="cuda:0")
    avl.avl_adjoint_push(sim.h, _t(x), _t(E), 1.0, ax, av, ax, av, Eb2)
    p = rng.permutation(n)
    out3 = [torch.empty(k, dtype=torch.float64, device="cuda:0") for k in (n, n, w.nx)]
    avl.avl_adjoint_push(sim.h, _t(x[p]), _t(E), 1.0, _t(lx1[p]), _t(lv1[p]), *out3)
    torch.cuda.synchronize()
    assert torch.equal(ax, out[0]) and torch.equal(av, out[1]) and torch.equal(Eb2, out[2])
    pt = torch.tensor(p, device="cuda:0")
    assert torch.equal(out3[0], out[0][pt]) and torch.equal(out3[1], out[1][pt])
    assert torch.equal(out3[2], out[2])


@pytest.mark.parametrize("precision", [avl.AVL_FP64, avl.AVL_FP32])
def test_deposit_stage_dot_product(precision):
    w, sim, g, rng = _case(precision)
    n = sim.n
    fg, D = sim.reconstruct(want_D=True)
    xs, vs, fs = sim.markers()
    rho_bar = rng.normal(size=w.nx)
    fb, lx, lv = (torch.empty(n, dtype=torch.float64, device="cuda:0") for _ in range(3))
    avl.avl_adjoint_deposit(sim.h, xs, vs.reshape(-1), fs, fg.contiguous(), D.contiguous(), _t(rho_bar), fb, lx, lv)
    torch.cuda.synchronize()
    xs, vs, fs = xs.cpu().numpy(), vs.cpu().numpy().reshape(-1), fs.cpu().numpy()
    fb, lx, lv = fb.cpu().numpy(), lx.cpu().numpy(), lv.cpu().numpy()
    tol = TOL if precision == avl.AVL_FP64 else 1e-5
    for trial in range(3):
        dx, dv, df = rng.normal(size=n), rng.normal(size=n), rng.normal(size=n)
        drho = tangent.deposit_tangent(g, xs, vs, fs, dx, dv, df)
        _check([drho * rho_bar], [df * fb, dx * lx, dv * lv], tol, f"deposit prec={precision} #{trial}")
    # weights only: the position adjoints are left out, f_bar is the same
    fb2 = torch.empty(n, dtype=torch.float64, device="cuda:0")
    avl.avl_adjoint_deposit(sim.h, _t(xs), _t(vs), _t(fs), fg.contiguous(), D.contiguous(), _t(rho_bar), fb2)
    torch.cuda.synchronize()
    assert np.array_equal(fb2.cpu().numpy(), fb)
    sim.check()


@pytest.mark.parametrize("nx", [8, 32, 1024])
def test_field_stage_dot_product(nx):
    w, sim, g, rng = _case(avl.AVL_FP64, nx=nx, nv=8, ppc=2)
    for trial in range(3):
        mu, drho = rng.normal(size=nx), rng.normal(size=nx)
        rb = torch.empty(nx, dtype=torch.float64, device="cuda:0")
        avl.avl_adjoint_field(sim.h, _t(mu), rb)
        torch.cuda.synchronize()
        rb = rb.cpu().numpy()
        dE = tangent.field_tangent(g, drho)
        _check([dE * mu], [drho * rb], TOL, f"field nx={nx} #{trial}")
    sim.check()


def test_stage_argument_errors():
    w, sim, g, rng = _case(avl.AVL_FP64, nx=16, nv=8, ppc=2)
    lib = avl.load()
    mu = _t(rng.normal(size=w.nx))
    assert lib.avl_adjoint_field(sim.h, mu.data_ptr(), mu.data_ptr()) == -1        # in place refused
    assert lib.avl_adjoint_field(sim.h, mu.data_ptr() + 4, mu.data_ptr()) == -3
    assert lib.avl_adjoint_push(sim.h, None, mu.data_ptr(), 1.0, None, None, None, None, mu.data_ptr()) == -1
    fb = torch.empty(sim.n, dtype=torch.float64, device="cuda:0")
    # exactly one of lam_x, lam_v given
    assert lib.avl_adjoint_deposit(sim.h, fb.data_ptr(), fb.data_ptr(), fb.data_ptr(), fb.data_ptr(), fb.data_ptr(),
                                   mu.data_ptr(), fb.data_ptr(), fb.data_ptr(), None) == -1
    w3 = inputs.two_stream_3v(nx=16, nv=4, ppc=1)
    x3, v3, f3 = inputs.markers(w3)
    s3 = avl.Simulation(w3, x3, v3.reshape(-1), f3)
    assert lib.avl_adjoint_push(s3.h, None, mu.data_ptr(), 1.0, None, None, None, None, mu.data_ptr()) == -6
    sim.check()
