"""Autotuner logic on the CPU (a fake timer) and on the GPU (a small case)."""
import os

import pytest

from paper_1804_03901_amd import avl, inputs, tune


def test_pick_takes_the_fastest_and_breaks_ties_low():
    times = {0: 3.0, 4: 2.0, 8: 2.0, 16: 5.0}
    best, table = tune.pick(list(times), lambda c: times[c], repeats=3)
    assert best == 4 and table == times


def test_shape_key_and_cache_round_trip(tmp_path):
    ws = inputs.batched_scan(count=2, seed=9, ppc=1, nx_choices=(16,), nv_choices=(8,))
    k1 = tune.shape_key(ws, avl.AVL_FP32)
    k2 = tune.shape_key(ws, avl.AVL_FP64)
    assert k1 != k2 and "1:16x8" in k1
    path = os.path.join(tmp_path, "t.json")
    tune._store_cache(path, {k1: {"rows": 6, "table": {"6": 1.0}}})
    assert tune._load_cache(path)[k1]["rows"] == 6
    assert tune._load_cache(os.path.join(tmp_path, "missing.json")) == {}


def test_search_is_coordinate_descent():
    # slot 0 best at 8 with the others at their defaults; slot 1 then best at 2
    cost = lambda t: abs(t[0] - 8) + (0 if t[1] == 2 else 1) + 0.5 * (t[0] == 8 and t[1] == 2)
    calls = []
    best, tables = tune.search([(0, (0, 4, 8)), (1, (0, 1, 2))], lambda t: calls.append(dict(t)) or cost(t),
                               repeats=1)
    assert best == {0: 8, 1: 2}
    assert set(tables) == {0, 1} and set(tables[0]) == {0, 4, 8} and set(tables[1]) == {0, 1, 2}
    # the second slot is searched with the first at its choice
    assert all(c[0] == 8 for c in calls[3:]) and all(c[1] == 0 for c in calls[:3])


def test_cache_entry_round_trip():
    best, tables = {0: 6, 1: 2, 2: 0}, {0: {0: 1.5, 6: 1.2}, 1: {0: 1.2, 2: 1.1}}
    e = tune._to_cache(best, tables)
    assert tune._from_cache(e) == (best, tables)


@pytest.mark.gpu
def test_tune_single_on_gpu(tmp_path):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    w = inputs.bump_on_tail(nx=256, nv=128, ppc=4, seed=2)
    path = os.path.join(tmp_path, "t.json")
    t, tables = tune.tune_single(w, candidates=(0, 4, 8), forms=(0, 1, 2), sort_blocks=(0, 2), steps=3, warmup=1,
                                 cache_path=path)
    assert t[avl.TUNE_RECON_ROWS] in (0, 4, 8) and set(tables[avl.TUNE_RECON_ROWS]) == {0, 4, 8}
    assert t[avl.TUNE_RECON_FORM] in (0, 1, 2) and set(tables[avl.TUNE_RECON_FORM]) == {0, 1, 2}
    assert t[avl.TUNE_SORT_BLOCKS] in (0, 2) and set(tables[avl.TUNE_SORT_BLOCKS]) == {0, 2}
    t2, tables2 = tune.tune_single(w, candidates=(0, 4, 8), cache_path=path)
    assert t2 == t and tables2 == tables


@pytest.mark.gpu
def test_tune_batch_on_gpu(tmp_path):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ws = inputs.batched_scan(count=3, seed=4, ppc=2, nx_choices=(32, 64), nv_choices=(16, 32))
    path = os.path.join(tmp_path, "t.json")
    ts, tables = tune.tune_batch(ws, candidates=(0, 4), forms=(1, 2), steps=2, warmup=1, cache_path=path)
    assert len(ts) == 3 and all(t == ts[0] for t in ts)
    assert set(tables) == {avl.TUNE_RECON_ROWS, avl.TUNE_RECON_FORM} and ts[0][avl.TUNE_RECON_FORM] in (1, 2)
