"""Bit-reproducibility of the step (the deterministic reduction of
Eq. (reconstruction)).

The sort's integer atomics order the markers inside each cell's run
differently from run to run; every run's sums are order-independent and all
sums above them have a fixed order, so f, D, rho, E and the per-step
diagnostics are a function of the marker multiset alone.  Checked here:
two independent runs, graph replay against direct launches, and a checkpoint
taken with avl_get_markers and loaded with avl_set_markers (FP64 form, whose
export is exact) against the uninterrupted run -- all bit for bit.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1804_03901_amd import avl, inputs

pytestmark = pytest.mark.gpu

CASES = {
    "ragged": inputs.bump_on_tail(nx=128, nv=100, ppc=7, seed=11),
    "stress": inputs.bump_on_tail(nx=256, nv=96, ppc=5, seed=12, weights="logu"),
    "landau": inputs.landau_small(),
}


def _sim(w, precision, markers=None):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    x, v, f = markers if markers is not None else inputs.markers(w)
    print(f"[case] {w.name} prec={precision} n={x.size}", flush=True)
    return avl.Simulation(w, x, v.reshape(-1), f, precision=precision)


def _state(sim):
    f, D = sim.reconstruct(want_D=True)
    E, rho = sim.field()
    torch.cuda.synchronize()
    return {"f": f.cpu().numpy(), "D": D.cpu().numpy(), "E": E.cpu().numpy(), "rho": rho.cpu().numpy()}


def _same(a, b, what):
    for k in a:
        assert np.array_equal(a[k].view(np.uint8), b[k].view(np.uint8)), f"{what}: {k} differs"


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("precision", [avl.AVL_FP64, avl.AVL_FP32])
def test_two_runs_bit_identical(case, precision):
    w = CASES[case]
    a = _sim(w, precision)
    b = _sim(w, precision)
    da = a.step(20).cpu().numpy()
    db = b.step(20).cpu().numpy()
    _same(_state(a), _state(b), "two runs")
    assert np.array_equal(da, db)
    # the marker multisets agree too (their storage order need not)
    xa, va, fa = (t.cpu().numpy() for t in a.markers())
    xb, vb, fb = (t.cpu().numpy() for t in b.markers())
    oa, ob = np.lexsort((fa, va[0], xa)), np.lexsort((fb, vb[0], xb))
    assert np.array_equal(xa[oa], xb[ob]) and np.array_equal(va[:, oa], vb[:, ob]) and np.array_equal(fa[oa], fb[ob])
    a.check()
    b.check()


@pytest.mark.parametrize("case", ["ragged", "stress"])
@pytest.mark.parametrize("precision", [avl.AVL_FP64, avl.AVL_FP32])
def test_graph_and_direct_bit_identical(case, precision):
    w = CASES[case]
    a = _sim(w, precision)
    b = _sim(w, precision)
    da = a.step(20, graph=False).cpu().numpy()
    db = b.step(20, graph=True).cpu().numpy()
    _same(_state(a), _state(b), "graph vs direct")
    assert np.array_equal(da, db)


@pytest.mark.parametrize("case", ["ragged", "landau"])
def test_checkpoint_resume_bit_identical(case):
    """FP64: 50 steps, export, load into a fresh handle, 50 more steps equals
    100 uninterrupted steps, bit for bit (fields, grid and diagnostics)."""
    w = CASES[case]
    whole = _sim(w, avl.AVL_FP64)
    d_whole = whole.step(100).cpu().numpy()
    first = _sim(w, avl.AVL_FP64)
    first.step(50)
    x, v, f = first.markers()
    resumed = _sim(w, avl.AVL_FP64, markers=(x.cpu().numpy(), v.cpu().numpy(), f.cpu().numpy()))
    d_res = resumed.step(50).cpu().numpy()
    _same(_state(whole), _state(resumed), "resume")
    assert np.array_equal(d_whole[50:], d_res)
    # and avl_set_markers on the first handle resumes the same way
    first.set_markers(x, v.reshape(-1), f)
    d_set = first.step(50).cpu().numpy()
    _same(_state(whole), _state(first), "set_markers resume")
    assert np.array_equal(d_whole[50:], d_set)


def test_permuted_load_bit_identical():
    """The same markers loaded in two different orders give the same grid,
    charge density and field, bit for bit, before and after steps."""
    w = CASES["stress"]
    x, v, f = inputs.markers(w)
    p = np.random.default_rng(5).permutation(x.size)
    for prec in (avl.AVL_FP64, avl.AVL_FP32):
        a = _sim(w, prec, markers=(x, v, f))
        b = _sim(w, prec, markers=(x[p], v[:, p], f[p]))
        _same(_state(a), _state(b), "permuted load")
        a.step(5)
        b.step(5)
        _same(_state(a), _state(b), "permuted load, 5 steps")


@pytest.mark.parametrize("case", ["ragged", "stress"])
def test_tuning_knobs_bit_identical(case):
    """The reconstruction's row form (dense or sparse register loads) and the
    sort passes' resident blocks change launch shapes only: after ten FP32
    steps f, D, rho, E and the diagnostics are the same bit for bit as with
    the library's defaults.  Rows per task regroups the rho partials, so at
    load f and D agree bit for bit and rho to rounding."""
    w = CASES[case]
    x, v, f = inputs.markers(w)

    def make(tune):
        if not torch.cuda.is_available():
            pytest.skip("no GPU")
        print(f"[case] {w.name} tune={tune}", flush=True)
        return avl.Simulation(w, x, v.reshape(-1), f, precision=avl.AVL_FP32, tune=tune)

    def run(tune):
        sim = make(tune)
        d = sim.step(10).cpu().numpy()
        s = _state(sim)
        sim.check()
        sim.close()
        return d, s

    d0, s0 = run(None)
    for t in ({avl.TUNE_RECON_FORM: 1}, {avl.TUNE_RECON_FORM: 2}, {avl.TUNE_SORT_BLOCKS: 1},
              {avl.TUNE_SORT_BLOCKS: 3, avl.TUNE_RECON_FORM: 1}):
        d, s = run(t)
        _same(s0, s, str(t))
        assert np.array_equal(d0, d), t
    a, b = make(None), make({avl.TUNE_RECON_ROWS: 3})
    sa, sb = _state(a), _state(b)
    for k in ("f", "D"):
        assert np.array_equal(sa[k].view(np.uint8), sb[k].view(np.uint8)), k
    assert np.max(np.abs(sa["rho"] - sb["rho"])) <= 1e-13 * np.max(np.abs(sa["rho"]))
    a.close()
    b.close()
