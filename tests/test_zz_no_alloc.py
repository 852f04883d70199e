"""avl_reconstruct_noalloc (the entry point for callers that cannot allocate)
against avl_init + avl_reconstruct on the same markers: bit for bit, on two
calls in a row (the second with fewer markers and a smaller grid, so stale
scratch contents from the first call would show), for both storage forms and
both velocity dimensionalities; and its refusal of a configuration past the
static array's size."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1804_03901_amd import avl, inputs

pytestmark = pytest.mark.gpu


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _reference(w, x, v, f, prec):
    sim = avl.Simulation(w, x, v.reshape(-1), f, precision=prec)
    fg, Dg = sim.reconstruct(want_D=True)
    torch.cuda.synchronize()
    sim.check()
    out = (fg.reshape(-1).clone(), Dg.reshape(-1).clone())
    sim.close()
    return out


def _noalloc(w, x, v, f, prec):
    dt = torch.float64 if prec == avl.AVL_FP64 else torch.float32
    dev = torch.device("cuda:0")
    xt = torch.tensor(x, dtype=torch.float64, device=dev)
    vt = torch.tensor(np.ascontiguousarray(v).reshape(-1), dtype=torch.float64, device=dev)
    ft = torch.tensor(f, dtype=torch.float64, device=dev)
    fo = torch.full((w.n_cells,), float("nan"), dtype=dt, device=dev)
    Do = torch.full((w.n_cells,), float("nan"), dtype=dt, device=dev)
    cfg = avl.make_config(w, prec, x.size)
    avl.avl_reconstruct_noalloc(cfg, torch.cuda.current_stream(), xt, vt, ft, fo, Do)
    torch.cuda.synchronize()
    return fo, Do


PAIRS = {
    "1v": (inputs.bump_on_tail(nx=256, nv=96, ppc=5, seed=12, weights="logu"),
           inputs.bump_on_tail(nx=64, nv=40, ppc=3, seed=31)),
    "1v_long_rows": (inputs.bump_on_tail(nx=64, nv=8, ppc=30, seed=14),
                     inputs.landau_small()),
    "3v": (inputs.two_stream_3v(nx=16, nv=8, ppc=2, seed=21),
           inputs.two_stream_3v(nx=8, nv=4, ppc=3, seed=22)),
}


@pytest.mark.parametrize("pair", list(PAIRS))
@pytest.mark.parametrize("prec", [avl.AVL_FP64, avl.AVL_FP32])
def test_noalloc_equals_handle_path(pair, prec):
    _gpu()
    for w in PAIRS[pair]:
        x, v, f = inputs.markers(w)
        print(f"[case] noalloc {w.name} prec={prec} n={x.size}", flush=True)
        f_ref, D_ref = _reference(w, x, v, f, prec)
        f_na, D_na = _noalloc(w, x, v, f, prec)
        assert torch.equal(f_na, f_ref), w.name
        assert torch.equal(D_na, D_ref), w.name


def test_noalloc_rejects_too_large_and_bad_arguments():
    _gpu()
    w = inputs.bump_on_tail()          # 16.8M markers: far past the static array
    cfg = avl.make_config(w, avl.AVL_FP32, w.n_markers)
    dev = torch.device("cuda:0")
    one = torch.zeros(8, dtype=torch.float64, device=dev)
    with pytest.raises(avl.AvlError) as e:
        avl.avl_reconstruct_noalloc(cfg, None, one, one, one, one)
    assert e.value.status == -2        # AVL_ESIZE
    small = inputs.landau_small()
    cfg = avl.make_config(small, avl.AVL_FP64, small.n_markers)
    with pytest.raises(avl.AvlError) as e:
        avl.avl_reconstruct_noalloc(cfg, None, one, one, one, None)
    assert e.value.status == -1        # AVL_EINVAL: no f_out
