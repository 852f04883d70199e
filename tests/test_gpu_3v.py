"""GPU parity of the 1D-3V path (16-cell cloud-in-cell volume weights) against
the FP64 CPU oracle, through the C ABI.

Same error measures as the 1D-1V tests (``checks``): normwise relative per
array, f also cell by cell where the oracle's weight sum is at least a tenth
of a marker, the field at its own scale max|E|.  FP64 path 1e-12 per step; FP32 form 1e-5 on
f.  The cases cover several 63-column strips with a ragged last strip, unequal
velocity resolutions per component, row segments too long to stage (the
reconstruction's global-memory path), and a one-strip grid whose periodic
wrap run exceeds a wavefront."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from checks import cell_rel, check_field, nrel
from paper_1804_03901_amd import avl, inputs

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL64_CELL = 1e-10


def t2n(t):
    return t.detach().double().cpu().numpy()


_base = inputs.two_stream_3v
CASES = {
    "cube": _base(nx=16, nv=8, ppc=2, seed=21),
    "strips": _base(nx=128, nv=8, ppc=2, seed=22).replace(name="ts3v_strips", nv=(12, 6, 4)),
    "long_rows": _base(nx=64, nv=4, ppc=12, seed=23).replace(name="ts3v_long_rows", nv=(4, 3, 3)),
    "wrap": _base(nx=8, nv=4, ppc=70, seed=24).replace(name="ts3v_wrap", nv=(3, 2, 2)),
}


def sim_for(w, precision=avl.AVL_FP64, markers=None):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    x, v, f = markers if markers is not None else inputs.markers(w)
    print(f"[case] {w.name} prec={precision} n={x.size}", flush=True)
    return avl.Simulation(w, x, v.reshape(-1), f, precision=precision), (x, v, f)


@pytest.mark.parametrize("case", list(CASES))
def test_3v_init_matches_oracle(case):
    w = CASES[case]
    sim, (x, v, f) = sim_for(w)
    g = oracle.Grid.from_workload(w)
    N, D, fo = oracle.reconstruct(g, x, v, f)
    rho_o, _, _ = oracle.moments(g, fo)
    E_o, _ = oracle.poisson(w.nx, w.L, w.c_p, rho_o)
    fg, Dg = sim.reconstruct(want_D=True)
    rho_g = sim.moments()
    E_g, _ = sim.poisson()
    sim.check()
    assert tuple(fg.shape) == (w.nv[2], w.nv[1], w.nv[0], w.nx)
    assert nrel(t2n(Dg), D) <= TOL64
    assert nrel(t2n(fg), fo) <= TOL64
    assert cell_rel(t2n(fg), fo, D) <= TOL64_CELL
    assert nrel(t2n(rho_g), rho_o) <= TOL64
    check_field(w, t2n(rho_g), t2n(E_g), rho_o, E_o, label=w.name)


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("graph", [False, True])
def test_3v_step_matches_oracle(case, graph):
    w = CASES[case]
    sim, _ = sim_for(w)
    sim.step(2, graph=graph)
    x, v, f = (t2n(a) for a in sim.markers())
    E = t2n(sim.field()[0])
    g = oracle.Grid.from_workload(w)
    xo, vo = oracle.push(g, x, v, E)
    _, Do, fo = oracle.reconstruct(g, xo, vo, f)
    rho_o, _, _ = oracle.moments(g, fo)
    E_o, _ = oracle.poisson(w.nx, w.L, w.c_p, rho_o)
    sim.step(1, graph=graph)
    fg, Dg = sim.reconstruct(want_D=True)
    E_g, rho_g = sim.field()
    sim.check()
    assert nrel(t2n(fg), fo) <= TOL64
    assert cell_rel(t2n(fg), fo, Do) <= TOL64_CELL
    assert nrel(t2n(Dg), Do) <= TOL64
    assert nrel(t2n(rho_g), rho_o) <= TOL64
    check_field(w, t2n(rho_g), t2n(E_g), rho_o, E_o, label=w.name)
    # the perpendicular velocities never change; x and vx match per marker
    # after pairing both sides by (vy, vz, x)
    xg, vg, _ = (t2n(a) for a in sim.markers())
    a = np.lexsort((xg, vg[2], vg[1]))
    b = np.lexsort((xo, vo[2], vo[1]))
    assert np.array_equal(vg[1:, a], vo[1:, b])
    dx = np.abs(xg[a] - xo[b])
    assert np.max(np.minimum(dx, w.L - dx)) <= TOL64 * w.L
    assert np.max(np.abs(vg[0, a] - vo[0, b])) <= TOL64 * (w.vmax[0] - w.vmin[0])


@pytest.mark.parametrize("case", ["cube", "strips", "long_rows"])
def test_3v_constant_f_is_reconstructed_exactly(case):
    """f = 1 on every marker gives N = D term by term, so f_g = 1 exactly
    wherever a cloud touches the cell (the paper's point about normalisation)."""
    w = CASES[case]
    x, v, _ = inputs.markers(w)
    sim, _ = sim_for(w, markers=(x, v, np.ones_like(x)))
    fg, Dg = sim.reconstruct(want_D=True)
    fg, Dg = t2n(fg), t2n(Dg)
    assert np.all(fg[Dg > 0] == 1.0)
    assert np.all(fg[Dg == 0] == 0.0)


@pytest.mark.parametrize("case", ["cube", "strips", "long_rows", "wrap"])
def test_3v_fp32_form_matches_oracle(case):
    w = CASES[case]
    sim, _ = sim_for(w, precision=avl.AVL_FP32)
    x, v, f = (t2n(a) for a in sim.markers())
    g = oracle.Grid.from_workload(w)
    _, D, fo = oracle.reconstruct(g, x, v, f)
    rho_o, _, _ = oracle.moments(g, fo)
    fg, Dg = sim.reconstruct(want_D=True)
    assert fg.dtype == torch.float32
    assert nrel(t2n(fg), fo) <= 1e-5
    assert cell_rel(t2n(fg), fo, D) <= 1e-5
    assert nrel(t2n(Dg), D) <= 1e-6
    assert nrel(t2n(sim.moments()), rho_o) <= 1e-6
    # one step from the exported state
    sim.step(2, graph=True)
    x, v, f = (t2n(a) for a in sim.markers())
    E = t2n(sim.field()[0])
    xo, vo = oracle.push(g, x, v, E)
    _, _, fo = oracle.reconstruct(g, xo, vo, f)
    rho_o, _, _ = oracle.moments(g, fo)
    E_o, _ = oracle.poisson(w.nx, w.L, w.c_p, rho_o)
    sim.step(1, graph=True)
    fg = sim.reconstruct()
    E_g, rho_g = sim.field()
    sim.check()
    assert nrel(t2n(fg), fo) <= 1e-5
    assert nrel(t2n(rho_g), rho_o) <= 1e-6
    check_field(w, t2n(rho_g), t2n(E_g), rho_o, E_o, label=w.name)



MAGNETISED = _base(nx=32, nv=8, ppc=2, seed=27).replace(name="ts3v_magnetised", nv=(10, 8, 6), B=(0.0, 0.3, 0.6))


@pytest.mark.parametrize("graph", [False, True])
def test_3v_magnetised_step_matches_oracle(graph):
    """Boris push with a background field across x and y: one step from the
    same exported state; all three velocity components now change, so the
    markers of both sides are paired by position."""
    w = MAGNETISED
    sim, _ = sim_for(w)
    sim.step(3, graph=graph)
    x, v, f = (t2n(a) for a in sim.markers())
    E = t2n(sim.field()[0])
    g = oracle.Grid.from_workload(w)
    xo, vo = oracle.push(g, x, v, E)
    _, Do, fo = oracle.reconstruct(g, xo, vo, f)
    rho_o, _, _ = oracle.moments(g, fo)
    E_o, _ = oracle.poisson(w.nx, w.L, w.c_p, rho_o)
    sim.step(1, graph=graph)
    fg, Dg = sim.reconstruct(want_D=True)
    E_g, rho_g = sim.field()
    sim.check()
    assert nrel(t2n(fg), fo) <= TOL64
    assert cell_rel(t2n(fg), fo, Do) <= TOL64_CELL
    assert nrel(t2n(Dg), Do) <= TOL64
    assert nrel(t2n(rho_g), rho_o) <= TOL64
    check_field(w, t2n(rho_g), t2n(E_g), rho_o, E_o, label=w.name)
    xg, vg, _ = (t2n(a) for a in sim.markers())
    a, b = np.argsort(xg), np.argsort(xo)
    assert np.max(np.abs(xg[a] - xo[b])) <= TOL64 * w.L
    assert np.max(np.abs(vg[:, a] - vo[:, b])) <= TOL64 * (w.vmax[0] - w.vmin[0])
    # the perpendicular velocities did turn
    assert np.max(np.abs(vo[1:] - v[1:])) > 1e-3


@pytest.mark.parametrize("precision", [avl.AVL_FP32, avl.AVL_FP64])
def test_full_size_two_stream_3v_sampled_planes(precision):
    """The 1D-3V benchmark workload at full size (nx = 512, 64^3 velocity
    cells, 4 markers per cell: 536,870,912 markers), in the FP32 form and in
    FP64, stepped as a replayed graph as the benchmark does.

    One step from the exported state is checked on sampled target (vy, vz)
    planes -- two corners of the velocity grid and an interior plane --
    against the oracle's push and reconstruction of the markers whose clouds
    reach those planes (selected from the exported state by their own vy, vz;
    without a magnetic field the push keeps both).  The charge density is
    checked on sampled x columns against the oracle's reconstruction and
    moments of every marker whose cloud reaches those columns (selected from
    the state the step left), and the field is the oracle's solve of the
    GPU's own rho at 1e-12 of max|E|, with W beside it.  Bounds: FP32 form 1e-5
    on f, 1e-6 on D and rho (normwise per plane, per column set); FP64 1e-12."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fp64 = precision == avl.AVL_FP64
    tol_f, tol_D, tol_rho = (TOL64, TOL64, TOL64) if fp64 else (1e-5, 1e-6, 1e-6)
    w = inputs.two_stream_3v()
    x, v, f = inputs.markers_threaded(w)
    print(f"[case] {w.name} prec={precision} n={x.size}", flush=True)
    sim = avl.Simulation(w, x, v.reshape(-1), f, precision=precision)
    del x, v, f
    sim.step(2, graph=True, diag=False)
    xt, vt, ft = sim.markers()
    E = t2n(sim.field()[0])
    planes = [(0, 0), (31, 17), (w.nv[1] - 1, w.nv[2] - 1)]
    # dual-plane indices of every marker's cloud in vy and vz
    jd = [torch.floor((vt[d] - w.vmin[d]) / ((w.vmax[d] - w.vmin[d]) / w.nv[d]) - 0.5) for d in (1, 2)]
    keep = torch.zeros_like(ft, dtype=torch.bool)
    for jy, jz in planes:
        keep |= ((jd[0] == jy - 1) | (jd[0] == jy)) & ((jd[1] == jz - 1) | (jd[1] == jz))
    xs, vs, fs = t2n(xt[keep]), t2n(vt[:, keep]), t2n(ft[keep])
    del xt, vt, ft, jd, keep
    print(f"[case] {xs.size} markers reach the sampled planes", flush=True)
    sim.step(1, graph=True, diag=False)
    fg, Dg = sim.reconstruct(want_D=True)
    fg, Dg = fg.reshape(w.nv[2], w.nv[1], w.nv[0], w.nx), Dg.reshape(w.nv[2], w.nv[1], w.nv[0], w.nx)
    g = oracle.Grid.from_workload(w)
    xo, vo = oracle.push(g, xs, vs, E)
    _, Do, fo = oracle.reconstruct(g, xo, vo, fs)
    del xo, vo, xs, vs, fs
    for jy, jz in planes:
        ef = nrel(t2n(fg[jz, jy]), fo[jz, jy])
        eD = nrel(t2n(Dg[jz, jy]), Do[jz, jy])
        print(f"[result] plane (vy {jy}, vz {jz}): f {ef:.2e} D {eD:.2e}", flush=True)
        assert ef <= tol_f
        assert eD <= tol_D
    del fg, Dg, fo, Do
    # rho on sampled columns: every marker whose x cloud reaches them
    E_g, rho_g = (t2n(a) for a in sim.field())
    cols = [0, 137, w.nx - 1]
    xt, vt, ft = sim.markers()
    ix = torch.floor(xt / (w.L / w.nx) - 0.5)
    ix = torch.where(ix < 0, ix + w.nx, ix)
    keep = torch.zeros_like(ft, dtype=torch.bool)
    for c in cols:
        # one dual cell of slack each way: a marker the selection takes in
        # excess only adds to columns that are not compared
        for d in (-2, -1, 0, 1):
            keep |= ix == (c + d) % w.nx
    xs, vs, fs = t2n(xt[keep]), t2n(vt[:, keep]), t2n(ft[keep])
    del xt, vt, ft, ix, keep
    print(f"[case] {xs.size} markers reach the sampled columns", flush=True)
    _, _, fo = oracle.reconstruct(g, xs, vs, fs)
    rho_o = oracle.moments(g, fo)[0][cols]
    del fo
    erho = float(np.max(np.abs(rho_g[cols] - rho_o)) / np.max(np.abs(rho_o)))
    print(f"[result] rho on columns {cols}: {erho:.2e}", flush=True)
    assert erho <= tol_rho
    # the field: the oracle's solve of the GPU's rho, and its energy
    E_o, _ = oracle.poisson(w.nx, w.L, w.c_p, rho_g)
    eE = float(np.max(np.abs(E_g - E_o)) / np.max(np.abs(E_o)))
    _, W_g = sim.poisson(None)
    W_g = float(t2n(W_g)[0])
    W_o = oracle.field_energy(w.nx, w.L, w.c_p, E_o)
    print(f"[result] E (solve of the GPU's rho) {eE:.2e} of max|E|; W {abs(W_g - W_o) / W_o:.2e}", flush=True)
    assert eE <= TOL64
    assert abs(W_g - W_o) <= TOL64 * W_o
    sim.check()
    sim.close()


def _edge_markers(w, off_grid):
    """Markers of w with groups moved onto the lower and upper cloud edges of
    each velocity axis (vmin - dv/2, vmax + dv/2, and just inside them) and,
    with off_grid, groups far outside in vy and vz; the moved markers carry
    the smallest weight present, so that the rounding of their edge weights
    is not magnified by a core weight.  Without off_grid the vy and vz edges
    are taken 1e-6 dv inside (an exact edge, or an offset within an FP32
    rounding of 1, may land outside, which the FP32 form cannot hold for those
    components; x-velocity clouds may leave the grid in both forms)."""
    x, v, f = inputs.markers(w)
    v, f = v.copy(), f.copy()
    k = 0
    for d in range(3):
        dv = (w.vmax[d] - w.vmin[d]) / w.nv[d]
        lo, hi = w.vmin[d] - 0.5 * dv, w.vmax[d] + 0.5 * dv
        if off_grid or d == 0:
            edges = [lo, np.nextafter(lo, np.inf), np.nextafter(hi, -np.inf), hi]
        else:
            edges = [lo + 1e-6 * dv, hi - 1e-6 * dv]
        for e in edges:
            v[d, k:k + 16] = e
            f[k:k + 16] = f.min()
            k += 16
    if off_grid:
        v[1, k:k + 16] = w.vmax[1] + 3.0      # outside in vy and vz: no weight anywhere
        v[2, k + 16:k + 32] = w.vmin[2] - 3.0
        f[k:k + 32] = f.min()
    return x, v, f


@pytest.mark.parametrize("precision", [avl.AVL_FP64, avl.AVL_FP32])
def test_3v_markers_on_velocity_grid_edges(precision):
    """Markers whose clouds end exactly on, or just inside, the edges of each
    velocity axis (and, in the FP64 form, vy and vz clouds off the grid),
    among ordinary markers: reconstruction, rho and one step against the
    oracle, every marker kept."""
    w = CASES["strips"]
    fp64 = precision == avl.AVL_FP64
    x, v, f = _edge_markers(w, off_grid=fp64)
    tol_f, tol_cell, tol_rho = (TOL64, TOL64_CELL, TOL64) if fp64 else (1e-5, 1e-5, 1e-6)
    sim, _ = sim_for(w, precision=precision, markers=(x, v, f))
    g = oracle.Grid.from_workload(w)
    xs, vs, fs = (t2n(a) for a in sim.markers())
    vs = vs.reshape(3, -1)
    _, D, fo = oracle.reconstruct(g, xs, vs, fs)
    fg, Dg = (t2n(a) for a in sim.reconstruct(want_D=True))
    assert nrel(fg, fo) <= tol_f and nrel(Dg, D) <= tol_f
    assert cell_rel(fg, fo, D) <= tol_cell
    E = t2n(sim.field()[0])
    xo, vo = oracle.push(g, xs, vs, E)
    _, Do, fo = oracle.reconstruct(g, xo, vo, fs)
    rho_o, _, _ = oracle.moments(g, fo)
    sim.step(1)
    fg, Dg = (t2n(a) for a in sim.reconstruct(want_D=True))
    _, rho_g = sim.field()
    print(f"[result] 3v velocity edges prec={precision}: f {nrel(fg, fo):.1e} cell {cell_rel(fg, fo, Do):.1e} "
          f"rho {nrel(t2n(rho_g), rho_o):.1e}", flush=True)
    # after an FP32 push the offsets of markers kicked off an x-velocity cloud
    # edge are tiny numbers held to FP32 absolute precision, so cells they
    # dominate carry that relative to their own f: normwise there, as in the
    # FP32 step test above; cell by cell for the FP64 path
    assert nrel(fg, fo) <= tol_f
    if fp64:
        assert cell_rel(fg, fo, Do) <= tol_cell
    assert nrel(t2n(rho_g), rho_o) <= tol_rho
    xg, vg, _ = (t2n(a) for a in sim.markers())
    assert xg.size == x.size
    vg = vg.reshape(3, -1)
    for d in range(3):
        tol_v = TOL64 * (w.vmax[d] - w.vmin[d]) if fp64 else 1e-5 * w.dv(d)
        assert np.max(np.abs(np.sort(vg[d]) - np.sort(vo[d]))) <= tol_v, d
    sim.check()


def test_3v_fp32_off_grid_vy_vz_is_reported():
    """The FP32 form cannot hold a vy or vz cloud off the velocity grid (those
    components never move, and the cell index has no room for them): such
    markers are stored in the overflow bucket, every kernel stays inside its
    arrays, and avl_check reports AVL_EINTERNAL, as the header states."""
    w = CASES["strips"]
    x, v, f = _edge_markers(w, off_grid=True)
    sim, _ = sim_for(w, precision=avl.AVL_FP32, markers=(x, v, f))
    sim.reconstruct()
    sim.step(2)
    torch.cuda.synchronize()
    with pytest.raises(avl.AvlError) as e:
        sim.check()
    assert e.value.status == -8
