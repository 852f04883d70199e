"""Autotuner for the library's kernel knobs (``avl_config.tune``).

Three knobs, searched one after another (coordinate descent, each with the
choices already made for the earlier ones):

* ``TUNE_RECON_ROWS``, the reconstruction's velocity rows per task: more rows
  mean fewer tasks, fewer re-read halo rows and fewer rho partials, fewer rows
  mean more tasks to fill the GPU;
* ``TUNE_RECON_FORM``, the FP32 reconstruction's row form: dense rows issue
  every register load of a row segment, sparse rows skip the loads past it
  (worth it when segments are well below the register capacity);
* ``TUNE_SORT_BLOCKS``, resident blocks per compute unit of the tiled count
  and scatter passes of a single FP32 instance (fewer blocks each walk more
  tiles; a batch's sort passes take a block per tile and ignore it).

The library picks defaults from the shape and the device; the tuner times
candidate values on the actual workload (a single instance or a batch), as
HIP-graph step replays, and keeps the fastest.  Choices are cached in a JSON
file keyed by the shapes, so a shape is timed once per machine.

Results never depend on the knobs beyond summation order, so any choice is
correct; only speed differs.
"""
from __future__ import annotations

import json
import os
import time
from typing import Callable, Optional, Sequence

from . import avl, inputs

DEFAULT_CANDIDATES = (0, 4, 6, 8, 10, 12, 16, 24)
FORM_CANDIDATES = (0, 1, 2)
SORT_BLOCK_CANDIDATES = (0, 2, 3, 4)
CACHE_VERSION = "v2"
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


def search(knobs, timer: Callable[[dict], float], repeats: int = 2):
    """Coordinate descent over ``knobs``, a list of (slot, candidates): each
    slot in turn takes the fastest of its candidates with the earlier slots
    fixed at their choices (0, the library default, for the later ones).
    Returns (tune dict, {slot: {candidate: ms}})."""
    chosen = {slot: 0 for slot, _ in knobs}
    tables = {}
    for slot, cands in knobs:
        best, tables[slot] = pick(cands, lambda c: timer({**chosen, slot: c}), repeats)
        chosen[slot] = best
    return chosen, tables


def _from_cache(entry):
    return ({int(k): v for k, v in entry["tune"].items()},
            {int(k): {int(c): ms for c, ms in t.items()} for k, t in entry["table"].items()})


def _to_cache(tune, tables):
    return {"tune": {str(k): v for k, v in tune.items()},
            "table": {str(k): {str(c): ms for c, ms in t.items()} for k, t in tables.items()}, "time": time.time()}


def tune_single(w: "inputs.Workload", markers=None, precision: int = avl.AVL_FP32, options: int = 0,
                candidates: Sequence[int] = DEFAULT_CANDIDATES, steps: int = 10, warmup: int = 3,
                cache_path: Optional[str] = CACHE_PATH, forms: Sequence[int] = FORM_CANDIDATES,
                sort_blocks: Sequence[int] = SORT_BLOCK_CANDIDATES):
    """Best ``tune`` dict for one instance, and the timing tables
    ({slot: {candidate: ms per step}}).  The row form and the sort blocks are
    searched only where they apply (FP32 1D-1V)."""
    key = f"{CACHE_VERSION}|single|" + shape_key([w], precision, options)
    cache = _load_cache(cache_path)
    if key in cache:
        return _from_cache(cache[key])
    x, v, f = markers if markers is not None else inputs.markers_threaded(w)

    def timer(t: dict) -> float:
        sim = avl.Simulation(w, x, v.reshape(-1), f, precision=precision, options=options, tune=t)
        try:
            return _graph_ms(lambda n: sim.step(n, graph=True, diag=False), sim.stream, steps, warmup)
        finally:
            sim.close()

    knobs = [(avl.TUNE_RECON_ROWS, tuple(candidates))]
    if precision == avl.AVL_FP32 and w.vdim == 1:
        knobs += [(avl.TUNE_RECON_FORM, tuple(forms)), (avl.TUNE_SORT_BLOCKS, tuple(sort_blocks))]
    best, tables = search([(s, c) for s, c in knobs if c], timer)
    cache[key] = _to_cache(best, tables)
    _store_cache(cache_path, cache)
    return best, tables


def tune_batch(workloads: Sequence["inputs.Workload"], markers=None, precision: int = avl.AVL_FP32,
               options: int = 0, candidates: Sequence[int] = DEFAULT_CANDIDATES, steps: int = 10,
               warmup: int = 3, cache_path: Optional[str] = CACHE_PATH, forms: Sequence[int] = FORM_CANDIDATES):
    """Best per-instance ``tune`` dicts for a batch (one value of each knob for
    all instances, 0 meaning each instance's own default), and the timing
    tables.  The batch's sort passes take a block per tile, so only the
    reconstruction's knobs are searched."""
    key = f"{CACHE_VERSION}|batch|" + shape_key(workloads, precision, options)
    cache = _load_cache(cache_path)
    if key in cache:
        best, tables = _from_cache(cache[key])
        return [dict(best) for _ in workloads], tables
    mk = markers if markers is not None else [inputs.markers_threaded(w) for w in workloads]

    def timer(t: dict) -> float:
        b = avl.Batch(workloads, mk, precision=precision, options=options, tunes=[t] * len(workloads))
        try:
            return _graph_ms(lambda n: b.step(n, diag=False), b.stream, steps, warmup)
        finally:
            b.close()

    knobs = [(avl.TUNE_RECON_ROWS, tuple(candidates))]
    if precision == avl.AVL_FP32:
        knobs.append((avl.TUNE_RECON_FORM, tuple(forms)))
    best, tables = search([(s, c) for s, c in knobs if c], timer)
    cache[key] = _to_cache(best, tables)
    _store_cache(cache_path, cache)
    return [dict(best) for _ in workloads], tables
