"""GPU parity of the FP32 form (cell index + FP32 offsets, FP32 f grid, FP64
rho and field solve) against the FP64 oracle.

Both sides start from the same state: the GPU's markers exported to FP64 (an
exact conversion of the stored cell + offsets).  Bounds: f within 1e-5
normwise relative per step and cell by cell where the oracle's weight sum is
at least a tenth of a marker (``checks.cell_rel``), the damping rate within 1%
of the oracle's.  The errors come from FP32 storage of offsets and f (relative
6e-8) and the FP32 products; the field is held to its own scale (``checks``).
A further test measures the whole error of the form, loading included, against
the oracle on the ORIGINAL FP64 markers."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from checks import cell_rel, check_field, nrel
from paper_1804_03901_amd import avl, inputs
from physics import damping_rate

pytestmark = pytest.mark.gpu

OPTIONS = {"fp64acc": 0, "kahan32": avl.AVL_OPT_KAHAN32}
TOL_F = 1e-5

CASES = {
    "landau": inputs.landau_small(),
    "ragged": inputs.bump_on_tail(nx=128, nv=100, ppc=7, seed=11),
    "stress": inputs.bump_on_tail(nx=256, nv=96, ppc=5, seed=12, weights="logu"),
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


def t2n(t):
    return t.detach().double().cpu().numpy()


def make(w, opt):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    x, v, f = inputs.markers(w)
    print(f"[case] {w.name} fp32 options={opt} n={x.size}", flush=True)
    return avl.Simulation(w, x, v.reshape(-1), f, precision=avl.AVL_FP32, options=opt), (x, v, f)


@pytest.mark.parametrize("opt", list(OPTIONS))
@pytest.mark.parametrize("case", list(CASES))
def test_fp32_reconstruction_of_exported_state(case, opt):
    w = CASES[case]
    sim, _ = make(w, OPTIONS[opt])
    x, v, f = (t2n(a) for a in sim.markers())
    g = oracle.Grid.from_workload(w)
    N, D, fo = oracle.reconstruct(g, x, v.reshape(1, -1), f)
    rho_o, _, _ = oracle.moments(g, fo)
    fg, Dg = sim.reconstruct(want_D=True)
    rho_g = sim.moments()
    sim.check()
    assert fg.dtype == torch.float32
    cell = cell_rel(t2n(fg), fo, D)
    print(f"[result] {case} {opt}: f {nrel(t2n(fg), fo):.2e} cell {cell:.2e} D {nrel(t2n(Dg), D):.2e}", flush=True)
    assert nrel(t2n(fg), fo) <= TOL_F
    assert cell <= TOL_F
    assert nrel(t2n(Dg), D) <= 1e-6
    assert nrel(t2n(rho_g), rho_o) <= 1e-6


@pytest.mark.parametrize("opt", list(OPTIONS))
@pytest.mark.parametrize("case", ["landau", "ragged", "stress"])
def test_fp32_error_from_original_markers(case, opt):
    """The FP32 form's whole error at load, against the oracle on the original
    FP64 markers: rounding of the offsets and of f to FP32 included."""
    w = CASES[case]
    sim, (x, v, f) = make(w, OPTIONS[opt])
    g = oracle.Grid.from_workload(w)
    N, D, fo = oracle.reconstruct(g, x, v, f)
    rho_o, _, _ = oracle.moments(g, fo)
    E_o, _ = oracle.poisson(w.nx, w.L, w.c_p, rho_o)
    fg, Dg = sim.reconstruct(want_D=True)
    E_g, rho_g = sim.field()
    sim.check()
    cell = cell_rel(t2n(fg), fo, D)
    r = check_field(w, t2n(rho_g), t2n(E_g), rho_o, E_o, label=f"{case} {opt}")
    print(f"[result] {case} {opt} from FP64 markers: f {nrel(t2n(fg), fo):.2e} cell {cell:.2e} "
          f"D {nrel(t2n(Dg), D):.2e} rho {nrel(t2n(rho_g), rho_o):.2e} E {r['E']:.2e}", flush=True)
    assert nrel(t2n(fg), fo) <= TOL_F
    assert cell <= TOL_F
    assert nrel(t2n(Dg), D) <= 1e-6
    assert nrel(t2n(rho_g), rho_o) <= 1e-6


@pytest.mark.parametrize("opt", list(OPTIONS))
@pytest.mark.parametrize("case", list(CASES))
def test_fp32_step_matches_oracle(case, opt):
    w = CASES[case]
    sim, _ = make(w, OPTIONS[opt])
    sim.step(3, graph=True)
    x, v, f = (t2n(a) for a in sim.markers())
    E, _ = sim.field()
    E = t2n(E)
    g = oracle.Grid.from_workload(w)
    xo, vo = oracle.push(g, x, v.reshape(1, -1), E)
    _, Do, fo = oracle.reconstruct(g, xo, vo, f)
    rho_o, _, _ = oracle.moments(g, fo)
    E_o, _ = oracle.poisson(w.nx, w.L, w.c_p, rho_o)
    d = t2n(sim.step(1, graph=True))
    fg = sim.reconstruct()
    E_g, rho_g = sim.field()
    sim.check()
    assert nrel(t2n(fg), fo) <= TOL_F
    assert cell_rel(t2n(fg), fo, Do) <= TOL_F
    assert nrel(t2n(rho_g), rho_o) <= 1e-6
    check_field(w, t2n(rho_g), t2n(E_g), rho_o, E_o, W_g=d[0, 0], label=f"{case} {opt}")
    # markers as multisets: compare the sorted marginals (pairing markers by a
    # sort on x would swap pairs closer than the FP32 offset resolution)
    xg, vg, _ = (t2n(a) for a in sim.markers())
    assert np.max(np.abs(np.sort(xg) - np.sort(xo))) <= 1e-5 * (w.L / w.nx)
    assert np.max(np.abs(np.sort(vg[0]) - np.sort(vo[0]))) <= 1e-5 * w.dv(0)


@pytest.mark.parametrize("opt", list(OPTIONS))
def test_fp32_landau_damping_rate(opt):
    w = CASES["landau"]
    sim, (x, v, f) = make(w, OPTIONS[opt])
    d = t2n(sim.step(w.steps, graph=True))
    sim.check()
    gam_g, _ = damping_rate(d[:, 1], w.dt)
    r = oracle.run(oracle.Grid.from_workload(w), x, v, f, w.steps)
    gam_o, _ = damping_rate(r["diag"][:, 1], w.dt)
    assert abs(gam_g - gam_o) <= 0.01 * abs(gam_o)
    # the field-energy history of the whole run against the FP64 oracle's
    W_g, W_o = d[:, 0], r["diag"][:, 0]
    dW = float(np.max(np.abs(W_g - W_o)) / np.max(W_o))
    print(f"[result] {opt}: damping rate {gam_g:.5f} (oracle {gam_o:.5f}), field energy history {dW:.2e}", flush=True)
    assert dW <= 1e-5


def test_fp32_export_round_trip():
    """Loading the exported FP32-form state again reproduces it exactly."""
    w = CASES["ragged"]
    sim, _ = make(w, 0)
    sim.step(4)
    x, v, f = sim.markers()
    E1, _ = sim.field()
    sim.set_markers(x, v.reshape(-1), f)
    x2, v2, f2 = sim.markers()
    sim.check()
    a = np.lexsort((t2n(v)[0], t2n(x)))
    b = np.lexsort((t2n(v2)[0], t2n(x2)))
    assert np.max(np.abs(t2n(x)[a] - t2n(x2)[b])) <= 1e-12 * w.L
    assert np.max(np.abs(t2n(v)[0][a] - t2n(v2)[0][b])) <= 1e-12 * w.dv(0)


def test_fp32_velocity_range_of_the_form():
    """The FP32 form holds velocity rows up to 2^(30 - log2 nx) - 2 from the
    grid: markers within that range are kept with their velocities (to FP32
    offset resolution); any finite velocity beyond it is clamped before the
    integer conversion and reported by avl_check (AVL_EINTERNAL), with no
    kernel leaving its arrays."""
    w = CASES["ragged"]
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    x, v, f = inputs.markers(w)
    dv = w.dv(0)
    lim_rows = 2 ** (30 - int(np.log2(w.nx))) - 2
    far_ok = np.array([w.vmax[0] + 0.5 * lim_rows * dv, w.vmin[0] - 0.5 * lim_rows * dv])
    v = v.copy()
    v[0, :2] = far_ok
    print(f"[case] {w.name} far velocities {far_ok}", flush=True)
    sim = avl.Simulation(w, x, v.reshape(-1), f, precision=avl.AVL_FP32)
    sim.step(2)
    sim.check()
    _, vg, _ = (t2n(a) for a in sim.markers())
    for u in far_ok:
        assert np.min(np.abs(vg[0] - u)) <= 1e-6 * abs(u), u
    sim.close()
    for bad in (1e30, -1e30, w.vmax[0] + 4.0 * lim_rows * dv):
        v2 = v.copy()
        v2[0, 5] = bad
        print(f"[case] {w.name} velocity {bad}", flush=True)
        sim = avl.Simulation(w, x, v2.reshape(-1), f, precision=avl.AVL_FP32)
        sim.step(1)
        torch.cuda.synchronize()
        with pytest.raises(avl.AvlError) as e:
            sim.check()
        assert e.value.status == -8
        sim.close()
