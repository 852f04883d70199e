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


@pytest.mark.gpu
def test_tune_single_on_gpu(tmp_path):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    w = inputs.bump_on_tail(nx=256, nv=128, ppc=4, seed=2)
    path = os.path.join(tmp_path, "t.json")
    t, table = tune.tune_single(w, candidates=(0, 4, 8), steps=3, warmup=1, cache_path=path)
    assert t[avl.TUNE_RECON_ROWS] in (0, 4, 8) and set(table) == {0, 4, 8}
    t2, _ = tune.tune_single(w, candidates=(0, 4, 8), cache_path=path)
    assert t2 == t
