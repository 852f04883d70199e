"""GPU parity of the HIP path against the FP64 CPU oracle, through the C ABI.

Every comparison starts both sides from the same exported state, so it checks
one stage or one step (trajectories of the full method are chaotic and are
compared through physics observables instead).  Error measure: normwise
relative, max|gpu - oracle| / max|oracle| per array (f, D, rho, marker
coordinates against their ranges), plus a cell-by-cell relative bound on f
wherever the oracle's weight sum D is above a floor; the field is checked at
its own scale, max|E| (``checks``).  FP64 path bound 1e-12 per step.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from checks import cell_rel, check_field, nrel
from paper_1804_03901_amd import avl, inputs
from physics import damping_rate, landau_root

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
# cell-wise f bound of the FP64 path where D_orc >= D_FLOOR.  A run's corner
# sums follow from its moment sums by differences, and each moment sum rounds
# its terms down onto a grid of about n 2^-51 of the run's largest |f| (the
# order-free sums); a cell whose own f is far below that of a neighbouring
# run it shares (log-uniform weights) sees that error relative to its own
# size: up to ~5e-12 measured on the stress case
TOL64_CELL = 1e-10


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def t2n(t):
    return t.detach().double().cpu().numpy()


def sim_for(w, precision=avl.AVL_FP64, markers=None):
    _need_gpu()
    x, v, f = markers if markers is not None else inputs.markers(w)
    print(f"[case] {w.name} prec={precision} n={x.size}", flush=True)
    return avl.Simulation(w, x, v.reshape(-1), f, precision=precision), (x, v, f)


CASES = {
    "landau": inputs.landau_small(),
    "ragged": inputs.bump_on_tail(nx=128, nv=100, ppc=7, seed=11),
    "tiny": inputs.landau_small().replace(name="tiny_nx8_nv2", nx=8, nv=(2, 1, 1), ppc=3),
    "stress": inputs.bump_on_tail(nx=256, nv=96, ppc=5, seed=12, weights="logu"),
    "wide_x": inputs.bump_on_tail(nx=1024, nv=16, ppc=6, seed=13),
    # row segments of about 63 x 30 markers, past what a reconstruction wave
    # stages in LDS (summed from global memory instead)
    "long_rows": inputs.bump_on_tail(nx=64, nv=8, ppc=30, seed=14).replace(name="long_rows_nx64_nv8_ppc30"),
    # one strip whose wrapped run (the column at x = L) exceeds a wavefront
    "wrap": inputs.bump_on_tail(nx=8, nv=4, ppc=80, seed=15).replace(name="wrap_nx8_nv4_ppc80"),
    # the largest grid the single-block field solve takes; the last of its 66
    # column strips holds one column.  (The FP32 form's x update adds b gamma,
    # gamma = dv dt / dx, in FP32, so its position error grows with gamma: here
    # about one cell per unit b, at the benchmark size 0.025.)
    "max_nx": inputs.bump_on_tail(nx=4096, nv=96, ppc=2, seed=16).replace(name="max_nx4096_nv96_ppc2"),
}


@pytest.mark.parametrize("case", list(CASES))
def test_init_reconstruct_moments_field(case):
    w = CASES[case]
    sim, (x, v, f) = sim_for(w)
    g = oracle.Grid.from_workload(w)
    N, D, fo = oracle.reconstruct(g, x, v, f)
    rho_o, _, _ = oracle.moments(g, fo)
    E_o, m1 = oracle.poisson(w.nx, w.L, w.c_p, rho_o)
    fg, Dg = sim.reconstruct(want_D=True)
    rho_g = sim.moments()
    E_g, W_g = sim.poisson()
    torch.cuda.synchronize()
    sim.check()
    assert nrel(t2n(Dg), D) <= TOL64
    assert nrel(t2n(fg), fo) <= TOL64
    assert nrel(t2n(rho_g), rho_o) <= TOL64
    assert cell_rel(t2n(fg), fo, D) <= TOL64_CELL
    check_field(w, t2n(rho_g), t2n(E_g), rho_o, E_o, W_g=t2n(W_g)[0], label=case)


@pytest.mark.parametrize("case", ["landau", "ragged", "tiny"])
def test_push_is_order_preserving_and_matches(case):
    w = CASES[case]
    sim, _ = sim_for(w)
    x0, v0, f0 = (t2n(a) for a in sim.markers())
    rng = np.random.default_rng(1)
    E = rng.normal(scale=0.3, size=w.nx)
    sim.push(torch.tensor(E, device="cuda:0"))
    x1, v1, f1 = (t2n(a) for a in sim.markers())
    g = oracle.Grid.from_workload(w)
    xo, vo = oracle.push(g, x0, v0, E)
    dx = np.abs(x1 - xo)
    dx = np.minimum(dx, w.L - dx)
    assert dx.max() <= TOL64 * w.L
    assert np.max(np.abs(v1 - vo)) <= TOL64 * (w.vmax[0] - w.vmin[0])
    assert np.array_equal(f1, f0)
    assert np.all((x1 >= 0) & (x1 < w.L))


def _one_step_oracle(w, x, v, f, E):
    g = oracle.Grid.from_workload(w)
    xo, vo = oracle.push(g, x, v, E)
    N, D, fo = oracle.reconstruct(g, xo, vo, f)
    rho, _, _ = oracle.moments(g, fo)
    En, m1 = oracle.poisson(w.nx, w.L, w.c_p, rho)
    return xo, vo, fo, D, rho, En, m1


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("graph", [False, True])
def test_full_step_matches_oracle(case, graph):
    w = CASES[case]
    sim, _ = sim_for(w)
    # take a few steps first so the state is not the loading order
    sim.step(3, graph=graph)
    x, v, f = (t2n(a) for a in sim.markers())
    E, _ = sim.field()
    E = t2n(E)
    xo, vo, fo, Do, rho_o, E_o, m1_o = _one_step_oracle(w, x, v.reshape(w.vdim, -1), f, E)
    d = t2n(sim.step(1, graph=graph))
    fg, Dg = sim.reconstruct(want_D=True)
    E_g, rho_g = sim.field()
    sim.check()
    assert nrel(t2n(fg), fo) <= TOL64
    assert nrel(t2n(Dg), Do) <= TOL64
    assert nrel(t2n(rho_g), rho_o) <= TOL64
    assert cell_rel(t2n(fg), fo, Do) <= TOL64_CELL
    Eg = t2n(E_g)
    r = check_field(w, t2n(rho_g), Eg, rho_o, E_o, W_g=d[0, 0], label=case)
    # mode-1 amplitude: within what the measured field difference allows
    dm1 = 2.0 / w.nx * np.sum(np.abs(Eg - E_o))
    assert abs(d[0, 1] - m1_o) <= dm1 * (1 + 1e-9) + TOL64 * np.max(np.abs(E_o))
    print(f"[result] {case} graph={graph}: f {nrel(t2n(fg), fo):.1e} cell {cell_rel(t2n(fg), fo, Do):.1e} "
          f"rho {nrel(t2n(rho_g), rho_o):.1e} E {r['E']:.1e} (bound {r['E_bound']:.1e}, solve {r['E_solve']:.1e})",
          flush=True)
    # markers: same multiset (compare sorted coordinates)
    xg, vg, fg_m = (t2n(a) for a in sim.markers())
    order_g = np.lexsort((vg[0], xg))
    order_o = np.lexsort((vo[0], xo))
    assert np.max(np.abs(xg[order_g] - xo[order_o])) <= TOL64 * w.L
    assert np.max(np.abs(vg[0][order_g] - vo[0][order_o])) <= TOL64 * (w.vmax[0] - w.vmin[0])
    assert np.array_equal(np.sort(fg_m), np.sort(f))


@pytest.mark.parametrize("case", ["ragged", "stress", "long_rows", "wrap"])
@pytest.mark.parametrize("precision", [avl.AVL_FP64, avl.AVL_FP32])
def test_constant_f_is_reconstructed_exactly(case, precision):
    """f = c on every marker (c a power of two) gives N = c D term by term, so
    f_g = c exactly wherever D > 0 (Eq. (reconstruction) reproduces a constant
    distribution whatever the marker positions), after steps too."""
    w = CASES[case]
    x, v, _ = inputs.markers(w)
    for c in (1.0, 0.25, 2.0 ** -30):
        sim, _ = sim_for(w, precision=precision, markers=(x, v, np.full(x.size, c)))
        for _ in range(2):
            fg, Dg = (t2n(a) for a in sim.reconstruct(want_D=True))
            assert np.all(fg[Dg > 0] == c) and np.all(fg[Dg == 0] == 0.0), c
            sim.step(2)
        sim.check()


def test_sorted_order_invariant():
    """After a step the exported markers are grouped by dual cell: the cell
    index is non-decreasing, and off-grid clouds come last."""
    w = CASES["ragged"]
    sim, _ = sim_for(w)
    sim.step(5)
    x, v, f = (t2n(a) for a in sim.markers())
    s = x / (w.L / w.nx) - 0.5
    i0 = np.floor(s).astype(np.int64) % w.nx
    t = (v[0] - w.vmin[0]) / w.dv(0) - 0.5
    j0 = np.floor(t).astype(np.int64)
    inside = (j0 >= -1) & (j0 <= w.nv[0] - 1)
    key = np.where(inside, (j0 + 1) * w.nx + i0, (w.nv[0] + 1) * w.nx)
    # floor decisions of the host may differ from the device's by one ulp at
    # cell edges; allow such markers, require order everywhere else
    edge = (np.abs(s - np.round(s)) < 1e-12) | (np.abs(t - np.round(t)) < 1e-12)
    dk = np.diff(key)
    assert np.all((dk >= 0) | edge[1:] | edge[:-1])


def test_empty_marker_set():
    w = inputs.landau_small().replace(name="empty")
    _need_gpu()
    e = np.zeros(0)
    sim = avl.Simulation(w, e, e, e)
    f = sim.reconstruct()
    E, rho = sim.field()
    d = sim.step(2)
    sim.check()
    assert float(f.abs().max()) == 0.0 if f.numel() else True
    assert float(E.abs().max()) == 0.0
    assert np.all(t2n(d) == 0.0)


def test_markers_outside_velocity_grid_are_kept():
    """Markers whose cloud misses the velocity grid contribute nothing but are
    still pushed and can come back."""
    w = inputs.landau_small().replace(name="outside")
    _need_gpu()
    x, v, f = inputs.markers(w)
    v = v.copy()
    v[0, :50] = 7.5     # above vmax + dv/2
    v[0, 50:100] = -9.0
    sim = avl.Simulation(w, x, v.reshape(-1), f)
    g = oracle.Grid.from_workload(w)
    N, D, fo = oracle.reconstruct(g, x, v, f)
    fg, Dg = sim.reconstruct(want_D=True)
    assert nrel(t2n(fg), fo) <= TOL64 and nrel(t2n(Dg), D) <= TOL64
    sim.step(2)
    xg, vg, _ = (t2n(a) for a in sim.markers())
    assert xg.size == x.size
    assert np.sum(vg[0] > 7.0) == 50 and np.sum(vg[0] < -8.5) == 50
    sim.check()


def test_landau_damping_on_gpu():
    """Landau case, 200 steps on the GPU: the damping rate agrees with the
    oracle run within 1% and with the exact root within 5%."""
    w = CASES["landau"]
    sim, (x, v, f) = sim_for(w)
    d = t2n(sim.step(w.steps, graph=True))
    gam_g, om_g = damping_rate(d[:, 1], w.dt)
    r = oracle.run(oracle.Grid.from_workload(w), x, v, f, w.steps)
    gam_o, om_o = damping_rate(r["diag"][:, 1], w.dt)
    root = landau_root(0.5)
    assert abs(gam_g - gam_o) <= 0.01 * abs(gam_o)
    assert abs(gam_g - root.imag) <= 0.05 * abs(root.imag)
    assert abs(om_g - root.real) <= 0.02 * root.real


def test_graph_and_direct_agree():
    """Graph replay and direct launches give the same run, bit for bit."""
    w = CASES["ragged"]
    a, _ = sim_for(w)
    b, _ = sim_for(w)
    da = t2n(a.step(20, graph=False))
    db = t2n(b.step(20, graph=True))
    Ea, rho_a = a.field()
    Eb, rho_b = b.field()
    assert torch.equal(Ea, Eb) and torch.equal(rho_a, rho_b)
    assert np.array_equal(da, db)


def test_set_markers_resume():
    """Checkpoint/resume: exporting the state after 10 steps and loading it
    into a new handle rebuilds exactly the field of the exported state."""
    w = CASES["landau"]
    a, _ = sim_for(w)
    a.step(10)
    x, v, f = a.markers()
    b, _ = sim_for(w)
    b.set_markers(x, v.reshape(-1), f)
    Ea, rho_a = a.field()
    Eb, rho_b = b.field()
    assert torch.equal(Ea, Eb) and torch.equal(rho_a, rho_b)


@pytest.mark.parametrize("precision,options,weights", [(avl.AVL_FP64, 0, "analytic"), (avl.AVL_FP32, 0, "analytic"),
                                                       (avl.AVL_FP32, avl.AVL_OPT_KAHAN32, "analytic"),
                                                       (avl.AVL_FP32, 0, "logu"),
                                                       (avl.AVL_FP32, avl.AVL_OPT_KAHAN32, "logu")])
def test_full_size_bump_on_tail_step(precision, options, weights):
    """The benchmark workload at full size (1024 x 1024 cells, 16 markers per
    cell, 16.8M markers), stepped as a replayed graph as the benchmark does:
    one step from the exported state against the oracle (FP64 path 1e-12,
    FP32 form, with FP64 or compensated FP32 sums, 1e-5 on f and 1e-6 on rho;
    the field at its own scale as everywhere).  Also with the configuration's
    log-uniform marker weights (1e-8 .. 1), the reconstruction's stress case."""
    w = inputs.bump_on_tail().replace(weights=weights)
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    x0, v0, f0 = inputs.markers(w)
    print(f"[case] {w.name} prec={precision} options={options} weights={weights} n={x0.size}", flush=True)
    sim = avl.Simulation(w, x0, v0.reshape(-1), f0, precision=precision, options=options)
    del x0, v0, f0
    tol_f, tol_r = (TOL64, TOL64) if precision == avl.AVL_FP64 else (1e-5, 1e-6)
    sim.step(2, graph=True, diag=False)
    x, v, f = (t2n(a) for a in sim.markers())
    E = t2n(sim.field()[0])
    xo, vo, fo, Do, rho_o, E_o, _ = _one_step_oracle(w, x, v.reshape(1, -1), f, E)
    sim.step(1, graph=True, diag=False)
    fg, Dg = sim.reconstruct(want_D=True)
    E_g, rho_g = sim.field()
    W_g = sim.diagnostics()["Ee"]
    sim.check()
    r = check_field(w, t2n(rho_g), t2n(E_g), rho_o, E_o, W_g=W_g, label=f"full size {precision}")
    cell = cell_rel(t2n(fg), fo, Do)
    print(f"[result] {precision} options={options} weights={weights}: f {nrel(t2n(fg), fo):.2e} cell {cell:.2e} D {nrel(t2n(Dg), Do):.2e} "
          f"rho {nrel(t2n(rho_g), rho_o):.2e} E {r['E']:.2e} (bound {r['E_bound']:.2e}, solve {r['E_solve']:.2e}) "
          f"W {r['W']:.2e}", flush=True)
    assert nrel(t2n(fg), fo) <= tol_f
    assert cell <= (TOL64_CELL if precision == avl.AVL_FP64 else tol_f)
    assert nrel(t2n(Dg), Do) <= tol_r
    assert nrel(t2n(rho_g), rho_o) <= tol_r


@pytest.mark.parametrize("precision", [avl.AVL_FP64, avl.AVL_FP32])
@pytest.mark.parametrize("weights", ["flat", "logu"])
def test_markers_on_grid_nodes(precision, weights):
    """One marker at every cell centre, where its cloud coincides with the
    cell (Eq. (reconstruction) with all weight on one corner), plus markers at
    x = 0 and just below x = L (the periodic wrap decided by rounding).  The
    oracle is matched; with weights within a factor of two (flat) every cell
    also returns its own marker's f, with D = 1."""
    _need_gpu()
    nx, nv = 64, 32
    w = inputs.bump_on_tail(nx=nx, nv=nv, ppc=1, seed=21).replace(name=f"nodes_{weights}")
    g = oracle.Grid.from_workload(w)
    dx, dv = w.L / nx, (w.vmax[0] - w.vmin[0]) / nv
    jj, ii = np.meshgrid(np.arange(nv), np.arange(nx), indexing="ij")
    x = ((ii + 0.5) * dx).ravel()
    v = (w.vmin[0] + (jj + 0.5) * dv).ravel()
    rng = np.random.default_rng(5)
    f = rng.uniform(0.5, 1.0, x.size) if weights == "flat" else np.exp(rng.uniform(np.log(1e-8), 0.0, x.size))
    # extra markers at the domain edges, weight zero-free but tiny, far from the nodes' f
    xe = np.array([0.0, np.nextafter(w.L, 0.0), w.L * (1 - 1e-15), 0.5 * dx])
    ve = w.vmin[0] + (np.array([3, 7, 11, 31]) + 0.5) * dv
    fe = np.full(4, 1e-3)
    x, v, f = np.concatenate([x, xe]), np.concatenate([v, ve]), np.concatenate([f, fe])
    sim, _ = sim_for(w, precision, markers=(x, v.reshape(1, -1), f))
    xs, vs, fs = (t2n(a) for a in sim.markers())
    N, D, fo = oracle.reconstruct(g, xs, vs.reshape(1, -1), fs)
    fg, Dg = (t2n(a) for a in sim.reconstruct(want_D=True))
    tol = TOL64 if precision == avl.AVL_FP64 else 1e-6
    print(f"[result] nodes {weights} prec={precision}: f {nrel(fg, fo):.2e} D {nrel(Dg, D):.2e} "
          f"cell {cell_rel(fg, fo, D):.2e}", flush=True)
    assert nrel(fg, fo) <= tol and nrel(Dg, D) <= tol
    if precision == avl.AVL_FP64 and weights == "logu":
        # A marker on a node is located by x (1/dx) here and by x / dx in the
        # oracle; the two may round to opposite sides of the node, which
        # moves a weight of the rounding of the cell coordinate (up to about
        # nx 2^-52 in x, nv 2^-52 in v) to the other neighbour.  A cell next
        # to a marker up to 1e8 times heavier sees that relative to its own
        # f, so the bound is 1e-12 of its f plus that weight times the
        # heaviest f its cloud neighbourhood holds (a dropped or misplaced
        # term would be of the order of f itself).
        fn = f[:nx * nv].reshape(nv, nx)
        nb = fn.copy()
        for dj in (-1, 0, 1):
            for di in (-1, 0, 1):
                sh = np.roll(fn, di, axis=1)
                sh = np.roll(sh, dj, axis=0) if dj else sh
                if dj == 1:
                    sh[0, :] = 0.0
                elif dj == -1:
                    sh[-1, :] = 0.0
                nb = np.maximum(nb, sh)
        nb = np.maximum(nb, fe.max())
        err = np.abs(fg - fo).reshape(nv, nx)
        bound = 1e-12 * np.abs(fo).reshape(nv, nx) + 4 * (nx + nv) * 2.0 ** -52 * nb
        print(f"[result] nodes logu: worst err / bound {np.max(err / bound):.2e}", flush=True)
        assert np.all(err <= bound)
    else:
        assert cell_rel(fg, fo, D) <= (TOL64_CELL if precision == avl.AVL_FP64 else 1e-5)
    if weights == "flat":
        # cells away from the extra markers: each holds its own marker alone
        own = np.ones((nv, nx), bool)
        for xv, vv in zip(xe, ve):
            i = int(np.floor(xv / dx)) % nx
            j = int(np.floor((vv - w.vmin[0]) / dv))
            own[max(j - 1, 0):j + 2, :] &= ~np.isin(np.arange(nx), [(i - 1) % nx, i, (i + 1) % nx])
        f_own = f[:nx * nv].reshape(nv, nx)
        if precision == avl.AVL_FP32:
            f_own = f_own.astype(np.float32).astype(np.float64)
        rel = np.abs(fg.reshape(nv, nx) - f_own) / f_own
        print(f"[result] nodes identity: max rel {rel[own].max():.2e}, D-1 {np.abs(Dg.reshape(nv, nx)[own] - 1).max():.2e}",
              flush=True)
        assert rel[own].max() <= (1e-13 if precision == avl.AVL_FP64 else 1e-6)
        assert np.abs(Dg.reshape(nv, nx)[own] - 1.0).max() <= (1e-13 if precision == avl.AVL_FP64 else 1e-6)
    sim.check()


@pytest.mark.parametrize("precision", [avl.AVL_FP64, avl.AVL_FP32])
def test_markers_on_velocity_grid_edges(precision):
    """Markers whose clouds end exactly on the edges of the velocity grid:
    at v = vmin - dv/2 (all weight on the row below the grid, lost), just
    inside it, just inside vmax + dv/2 and exactly on it (the overflow
    bucket; in the FP32 form those keep stored cell indices), among ordinary
    markers; reconstruction and one step against the oracle, and every
    marker kept.  FP32 form: the FP32 push's bounds (1e-5 on f, offsets to
    1e-5 of a cell)."""
    w = CASES["ragged"]
    _need_gpu()
    fp64 = precision == avl.AVL_FP64
    tol_f, tol_cell, tol_rho = (TOL64, TOL64_CELL, TOL64) if fp64 else (1e-5, 1e-5, 1e-6)
    x, v, f = inputs.markers(w)
    v = v.copy()
    dv = (w.vmax[0] - w.vmin[0]) / w.nv[0]
    lo, hi = w.vmin[0] - 0.5 * dv, w.vmax[0] + 0.5 * dv
    edge = np.array([lo, np.nextafter(lo, np.inf), lo + 1e-9 * dv, np.nextafter(hi, -np.inf), hi - 1e-9 * dv, hi])
    k = np.arange(edge.size * 20)
    v[0, k] = np.repeat(edge, 20)
    # weights of the tail they now sit in (the smallest present), so that the
    # rounding of their tiny edge weights is not magnified by a core weight
    f = f.copy()
    f[k] = f.min()
    sim, _ = sim_for(w, precision=precision, markers=(x, v, f))
    g = oracle.Grid.from_workload(w)
    xs, vs, fs = (t2n(a) for a in sim.markers())
    N, D, fo = oracle.reconstruct(g, xs, vs.reshape(1, -1), fs)
    fg, Dg = (t2n(a) for a in sim.reconstruct(want_D=True))
    assert nrel(fg, fo) <= tol_f and nrel(Dg, D) <= tol_f
    assert cell_rel(fg, fo, D) <= tol_cell
    E, _ = sim.field()
    xo, vo, fo1, Do1, rho_o, _, _ = _one_step_oracle(w, xs, vs.reshape(1, -1), fs, t2n(E))
    sim.step(1)
    fg, Dg = (t2n(a) for a in sim.reconstruct(want_D=True))
    _, rho_g = sim.field()
    print(f"[result] velocity edges prec={precision}: f {nrel(fg, fo1):.1e} cell {cell_rel(fg, fo1, Do1):.1e} "
          f"rho {nrel(t2n(rho_g), rho_o):.1e}", flush=True)
    assert nrel(fg, fo1) <= tol_f and nrel(Dg, Do1) <= tol_f
    assert cell_rel(fg, fo1, Do1) <= tol_cell
    assert nrel(t2n(rho_g), rho_o) <= tol_rho
    xg, vg, _ = (t2n(a) for a in sim.markers())
    assert xg.size == x.size
    if fp64:
        og, oo = np.lexsort((vg[0], xg)), np.lexsort((vo[0], xo))
        assert np.max(np.abs(vg[0][og] - vo[0][oo])) <= TOL64 * (w.vmax[0] - w.vmin[0])
    else:
        assert np.max(np.abs(np.sort(vg[0]) - np.sort(vo[0]))) <= 1e-5 * w.dv(0)
    sim.check()


@pytest.mark.parametrize("precision", [avl.AVL_FP64, avl.AVL_FP32])
def test_zero_and_signed_weights(precision):
    """All weights zero: every run's largest |f| is zero, f_g = 0 exactly and D
    is unchanged.  Weights of both signs (a perturbation-like f): the sums
    round every term down onto their grid whatever its sign; against the
    oracle normwise, and cell by cell where |f| is not cancelled below a
    thousandth of its largest value."""
    w = CASES["ragged"]
    x, v, _ = inputs.markers(w)
    g = oracle.Grid.from_workload(w)
    tol = TOL64 if precision == avl.AVL_FP64 else 1e-5
    sim, _ = sim_for(w, precision=precision, markers=(x, v, np.zeros(x.size)))
    fg, Dg = (t2n(a) for a in sim.reconstruct(want_D=True))
    xs, vs, fs = (t2n(a) for a in sim.markers())
    _, D, _ = oracle.reconstruct(g, xs, vs.reshape(1, -1), fs)
    assert np.all(fg == 0.0) and nrel(Dg, D) <= tol
    sim.step(2)
    assert np.all(t2n(sim.reconstruct()) == 0.0)
    sim.check()
    rng = np.random.default_rng(3)
    f = rng.normal(size=x.size) * np.exp(rng.uniform(-6.0, 0.0, x.size))
    sim, _ = sim_for(w, precision=precision, markers=(x, v, f))
    xs, vs, fs = (t2n(a) for a in sim.markers())
    _, D, fo = oracle.reconstruct(g, xs, vs.reshape(1, -1), fs)
    fg, Dg = (t2n(a) for a in sim.reconstruct(want_D=True))
    m = (D >= 0.1) & (np.abs(fo) >= 1e-3 * np.max(np.abs(fo)))
    rel = np.max(np.abs(fg[m] - fo[m]) / np.abs(fo[m]))
    print(f"[result] signed weights prec={precision}: f {nrel(fg, fo):.1e} cell {rel:.1e}", flush=True)
    assert nrel(fg, fo) <= tol and nrel(Dg, D) <= tol
    assert rel <= (1e-10 if precision == avl.AVL_FP64 else 1e-4)
    sim.check()


@pytest.mark.parametrize("precision", [avl.AVL_FP64, avl.AVL_FP32])
def test_large_kicks_step(precision):
    """A strongly perturbed plasma on a coarse step (density 1 + 0.9 cos kx,
    dt = 2, 256 velocity cells): kicks of over ten velocity cells and drifts
    of tens of x cells a step, so many markers land outside the sort's LDS
    window and take its one-slot-at-a-time path.  One step against the
    oracle from the exported state (FP32 form: its push's bounds)."""
    w = inputs.landau_small().replace(name="large_kicks", mode_amplitude=0.9, dt=2.0, nv=(256, 1, 1))
    fp64 = precision == avl.AVL_FP64
    sim, _ = sim_for(w, precision=precision)
    # the first step: the loaded field is the strongest (plasma oscillation)
    x, v, f = (t2n(a) for a in sim.markers())
    E = t2n(sim.field()[0])
    dv = w.dv(0)
    kick = np.max(np.abs(E)) * w.dt / dv
    print(f"[case] large kicks: max |kick| {kick:.1f} cells", flush=True)
    assert kick > 8.0
    xo, vo, fo, Do, rho_o, _, _ = _one_step_oracle(w, x, v.reshape(1, -1), f, E)
    sim.step(1)
    fg, Dg = (t2n(a) for a in sim.reconstruct(want_D=True))
    _, rho_g = sim.field()
    tol_f, tol_rho = (TOL64, TOL64) if fp64 else (1e-5, 1e-6)
    print(f"[result] large kicks prec={precision}: f {nrel(fg, fo):.1e} cell {cell_rel(fg, fo, Do):.1e} "
          f"rho {nrel(t2n(rho_g), rho_o):.1e}", flush=True)
    assert nrel(fg, fo) <= tol_f and nrel(Dg, Do) <= tol_f
    assert cell_rel(fg, fo, Do) <= (TOL64_CELL if fp64 else 1e-5)
    assert nrel(t2n(rho_g), rho_o) <= tol_rho
    xg, vg, _ = (t2n(a) for a in sim.markers())
    if fp64:
        og, oo = np.lexsort((vg[0], xg)), np.lexsort((vo[0], xo))
        assert np.max(np.abs(xg[og] - xo[oo])) <= TOL64 * w.L
        assert np.max(np.abs(vg[0][og] - vo[0][oo])) <= TOL64 * (w.vmax[0] - w.vmin[0])
    else:
        # the FP32 offset update b + e rounds at the FP32 spacing of |e|, the
        # kick in cells: K 2^-23 of a cell for a kick of K cells
        assert np.max(np.abs(np.sort(vg[0]) - np.sort(vo[0]))) <= (1e-5 + 4 * kick * 2.0 ** -24) * dv
    sim.check()


@pytest.mark.parametrize("precision", [avl.AVL_FP64, avl.AVL_FP32])
def test_long_overflow_run_step(precision):
    """A third of the markers outside the velocity grid, above and below it:
    their run (the overflow bucket, stored cell indices in the FP32 form) spans
    many sort tiles, so whole count and scatter tiles lie past its start.  One
    step against the oracle from the exported state, then more steps keep
    every marker and the multiset of weights (FP32 form: its push's bounds)."""
    w = CASES["ragged"]
    _need_gpu()
    fp64 = precision == avl.AVL_FP64
    x, v, f = inputs.markers(w)
    v = v.copy()
    dv = w.dv(0)
    rng = np.random.default_rng(71)
    out = rng.random(x.size) < 1.0 / 3.0
    up = rng.random(x.size) < 0.5
    spread = 2.0 + 20.0 * rng.random(x.size)
    v[0] = np.where(out & up, w.vmax[0] + spread * dv, np.where(out, w.vmin[0] - spread * dv, v[0]))
    sim, _ = sim_for(w, precision=precision, markers=(x, v, f))
    n_out = int(out.sum())
    print(f"[case] long overflow run: {n_out} of {x.size} markers outside", flush=True)
    assert n_out > 4 * 4096
    xs, vs, fs = (t2n(a) for a in sim.markers())
    E = t2n(sim.field()[0])
    xo, vo, fo, Do, rho_o, _, _ = _one_step_oracle(w, xs, vs.reshape(1, -1), fs, E)
    sim.step(1)
    fg, Dg = (t2n(a) for a in sim.reconstruct(want_D=True))
    _, rho_g = sim.field()
    tol_f, tol_rho = (TOL64, TOL64) if fp64 else (1e-5, 1e-6)
    print(f"[result] long overflow run prec={precision}: f {nrel(fg, fo):.1e} cell {cell_rel(fg, fo, Do):.1e} "
          f"rho {nrel(t2n(rho_g), rho_o):.1e}", flush=True)
    assert nrel(fg, fo) <= tol_f and nrel(Dg, Do) <= tol_f
    assert cell_rel(fg, fo, Do) <= (TOL64_CELL if fp64 else 1e-5)
    assert nrel(t2n(rho_g), rho_o) <= tol_rho
    xg, vg, _ = (t2n(a) for a in sim.markers())
    kick = np.max(np.abs(E)) * w.dt / dv
    assert np.max(np.abs(np.sort(vg[0]) - np.sort(vo[0]))) <= (TOL64 * (w.vmax[0] - w.vmin[0]) if fp64 else
                                                            (1e-5 + 4 * kick * 2.0 ** -24) * dv)
    sim.step(4)
    xg, vg, fg1 = (t2n(a) for a in sim.markers())
    assert xg.size == x.size
    assert np.array_equal(np.sort(fg1), np.sort(fs))
    assert np.sum((vg[0] > w.vmax[0] + dv) | (vg[0] < w.vmin[0] - dv)) > 4 * 4096
    sim.check()
