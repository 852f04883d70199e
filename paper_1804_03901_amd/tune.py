"""Autotuner for the library's kernel knobs (``avl_config.tune``).

The knob that matters is the reconstruction's rows per task (slot
``TUNE_RECON_ROWS``): more rows per task mean fewer tasks, fewer re-read halo
rows and fewer rho partials, fewer rows mean more tasks to fill the GPU.  The
library picks a default from the shape and the device; the tuner times
candidate values on the actual workload (a single instance or a batch), as
HIP-graph step replays, and keeps the fastest.  Choices are cached in a JSON
file keyed by the shapes, so a shape is timed once per machine.

Results never depend on the knob beyond summation order, so any choice is
correct; only speed differs.
"""
from __future__ import annotations

import json
import os
import time
from typing import Callable, Optional, Sequence

from . import avl, inputs

DEFAULT_CANDIDATES = (0, 4, 6, 8, 10, 12, 16, 24)
CACHE_PATH = os.path.join(os.path.expanduser("~"), ".cache", "avl", "tune.json")


def shape_key(workloads: Sequence["inputs.Workload"], precision: int, options: int = 0) -> str:
    """Cache key: precision, options and the (nx, nv, markers) of every instance."""
    parts = [f"p{precision}o{options}"]
    for w in workloads:
        parts.append(f"{w.vdim}:{w.nx}x{'x'.join(str(n) for n in w.nv[: w.vdim])}:{w.n_markers}")
    return "|".join(parts)


def _load_cache(path: Optional[str]) -> dict:
    if not path or not os.path.exists(path):
        return {}
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store_cache(path: Optional[str], cache: dict) -> None:
    if not path:
        return
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = f"{path}.{os.getpid()}"
    with open(tmp, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def pick(candidates: Sequence[int], timer: Callable[[int], float], repeats: int = 2):
    """Time every candidate (best of ``repeats``) and return (best, {candidate: ms})."""
    table = {}
    for c in candidates:
        table[c] = min(timer(c) for _ in range(repeats))
    best = min(table, key=lambda c: (table[c], c))
    return best, table


def _graph_ms(run_steps, stream, steps: int, warmup: int) -> float:
    import torch
    run_steps(warmup)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record(stream)
    run_steps(steps)
    t1.record(stream)
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) / steps


def tune_single(w: "inputs.Workload", markers=None, precision: int = avl.AVL_FP32, options: int = 0,
                candidates: Sequence[int] = DEFAULT_CANDIDATES, steps: int = 10, warmup: int = 3,
                cache_path: Optional[str] = CACHE_PATH):
    """Best ``tune`` dict for one instance, and the timing table (ms per step)."""
    key = "single|" + shape_key([w], precision, options)
    cache = _load_cache(cache_path)
    if key in cache:
        return {avl.TUNE_RECON_ROWS: cache[key]["rows"]}, cache[key]["table"]
    x, v, f = markers if markers is not None else inputs.markers_threaded(w)

    def timer(rows: int) -> float:
        sim = avl.Simulation(w, x, v.reshape(-1), f, precision=precision, options=options,
                             tune={avl.TUNE_RECON_ROWS: rows})
        try:
            return _graph_ms(lambda n: sim.step(n, graph=True, diag=False), sim.stream, steps, warmup)
        finally:
            sim.close()

    best, table = pick(candidates, timer)
    cache[key] = {"rows": best, "table": {str(k): v for k, v in table.items()}, "time": time.time()}
    _store_cache(cache_path, cache)
    return {avl.TUNE_RECON_ROWS: best}, table


def tune_batch(workloads: Sequence["inputs.Workload"], markers=None, precision: int = avl.AVL_FP32,
               options: int = 0, candidates: Sequence[int] = DEFAULT_CANDIDATES, steps: int = 10,
               warmup: int = 3, cache_path: Optional[str] = CACHE_PATH):
    """Best per-instance ``tune`` dicts for a batch (one rows value for all
    instances, 0 meaning each instance's own default), and the timing table."""
    key = "batch|" + shape_key(workloads, precision, options)
    cache = _load_cache(cache_path)
    if key in cache:
        rows = cache[key]["rows"]
        return [{avl.TUNE_RECON_ROWS: rows}] * len(workloads), cache[key]["table"]
    mk = markers if markers is not None else [inputs.markers_threaded(w) for w in workloads]

    def timer(rows: int) -> float:
        b = avl.Batch(workloads, mk, precision=precision, options=options,
                      tunes=[{avl.TUNE_RECON_ROWS: rows}] * len(workloads))
        try:
            return _graph_ms(lambda n: b.step(n, diag=False), b.stream, steps, warmup)
        finally:
            b.close()

    best, table = pick(candidates, timer)
    cache[key] = {"rows": best, "table": {str(k): v for k, v in table.items()}, "time": time.time()}
    _store_cache(cache_path, cache)
    return [{avl.TUNE_RECON_ROWS: best}] * len(workloads), table
