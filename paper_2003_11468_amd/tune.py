"""Autotuner for the two launch parameters of the labelling pipeline.

- cell_factor: cell side in units of l_x (>= 1; 0 = about one particle per
  cell). Smaller cells test fewer pairs inside dense groups but cost more
  cell bookkeeping; the best value depends on the clustering.
- dense_min: cells with at least this many particles are searched by whole
  wavefronts (64 particles against broadcast candidates), the others by the
  load-balanced per-particle search.

Every candidate runs the full pipeline (build, link, finalize) on the caller's
own input, timed with HIP events on the stream it runs on; the fastest wins.
Results are cached in a JSON file keyed by the workload class: predicate,
particle count and box count rounded to powers of two, and the median
dimensionless linking length b = l_x n^(1/3) / L. Any candidate gives the same
labels, so tuning never changes a result, only the time.
"""
from __future__ import annotations

import json
import math
import os
import statistics

import numpy as np

from . import FoF, FoFError, fof_build_cells, fof_finalize, fof_link

CELL_FACTORS = (0.0, 1.5, 2.0, 2.5, 3.0, 4.0)
DENSE_MINS = (8, 16, 32)
DEFAULT_CACHE = os.environ.get("FOF_TUNE_CACHE",
                               os.path.join(os.path.expanduser("~"), ".cache", "paper_2003_11468_amd", "tune.json"))


def workload_key(offsets, box, lx, predicate: str, strict: bool = False) -> str:
    off = np.asarray(offsets, dtype=np.int64)
    sizes = np.diff(off)
    n = int(off[-1])
    L = np.broadcast_to(np.asarray(box, dtype=np.float64), sizes.shape)
    l = np.broadcast_to(np.asarray(lx, dtype=np.float64), sizes.shape)
    keep = sizes > 0
    b = float(np.median(l[keep] * np.cbrt(sizes[keep].astype(np.float64)) / L[keep])) if keep.any() else 0.0
    return "%s|%s|n2^%d|boxes2^%d|b%.2g" % (predicate, "lt" if strict else "le", round(math.log2(max(n, 1))),
                                           round(math.log2(max(len(sizes), 1))), b)


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save(path, cache):
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def time_config(torch, pos, offsets, box, lx, predicate, strict, cell_factor, dense_min, repeats=3,
                max_workspace=None):
    """Median ms of build+link+finalize for one configuration (None if it cannot run)."""
    f = FoF(predicate, strict, cell_factor, dense_min=dense_min)
    try:
        try:
            from . import fof_workspace_bytes

            need = fof_workspace_bytes(f.ctx, offsets, box, lx)
        except FoFError:
            return None
        if max_workspace is not None and need > max_workspace:
            return None
        f.reserve(offsets, box, lx)
        label, size = f.outputs(pos.shape[0])
        times = []
        for rep in range(repeats + 1):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(f.stream)
            fof_build_cells(f.ctx, pos, offsets, box, lx)
            fof_link(f.ctx)
            fof_finalize(f.ctx, label, size)
            e1.record(f.stream)
            e1.synchronize()
            if rep:
                times.append(e0.elapsed_time(e1))
        return statistics.median(times)
    finally:
        f.close()


def autotune(pos, offsets, box, lx, predicate: str = "fp32_filter", strict: bool = False,
             cache_path: str | None = DEFAULT_CACHE, repeats: int = 3, cell_factors=CELL_FACTORS,
             dense_mins=DENSE_MINS, max_workspace: int | None = None, force: bool = False) -> dict:
    """Returns {"cell_factor", "dense_min", "ms", "key", "tried"} for this workload class."""
    import torch

    key = workload_key(offsets, box, lx, predicate, strict)
    cache = _load(cache_path) if cache_path else {}
    if not force and key in cache:
        return dict(cache[key], key=key, cached=True)
    if max_workspace is None:
        free, _ = torch.cuda.mem_get_info(pos.device)
        max_workspace = free // 2
    tried = []
    for cf in cell_factors:
        for dm in dense_mins:
            ms = time_config(torch, pos, offsets, box, lx, predicate, strict, cf, dm, repeats, max_workspace)
            tried.append({"cell_factor": cf, "dense_min": dm, "ms": ms})
    ok = [t for t in tried if t["ms"] is not None]
    if not ok:
        raise RuntimeError("no configuration could run")
    best = min(ok, key=lambda t: t["ms"])
    out = {"cell_factor": best["cell_factor"], "dense_min": best["dense_min"], "ms": best["ms"], "tried": tried}
    if cache_path:
        cache = _load(cache_path)
        cache[key] = out
        _save(cache_path, cache)
    return dict(out, key=key, cached=False)
