"""Autotuner for the launch parameters of the labelling pipeline.

Cell size and tile shape:
- cell_factor: cell side in units of l_x (>= 1; 0 = about one particle per
  cell). Smaller cells test fewer pairs inside dense groups but cost more
  cell bookkeeping; the best value depends on the clustering.
- dense_min: cells with at least this many particles are searched by whole
  wavefronts (tiles of 64 home particles against 64 staged candidates), the
  others by the load-balanced per-particle search (tiles of 64 home
  particles, each with its own candidate ranges).
- segment_log2: cells per work-group of the in-LDS cell sort (0: automatic).
Work schedule and contention variants:
- schedule: work-groups of the two persistent link kernels, whether dense
  cells are pre-merged by sub-cells, the giant-component skip, and whether
  the per-particle search joins the links inside its tiles
  (fof_options.schedule);
- link_order: hook by index or by a pseudo-random priority (paper, Section 3.2);
- compression: path halving or compression of paths of length >= 2 only
  (paper, Section 3.4.3).

Search: the full grid of cell_factor x dense_min first, then one axis at a
time (coordinate descent) over the others, each candidate keeping the best
values so far. Every candidate runs the full pipeline (build, link,
finalize) on the caller's own input, timed with HIP events on the stream it
runs on; the fastest wins. Results are cached in a JSON file keyed by the
workload class: predicate, GPU architecture, particle and box counts rounded
to powers of two, the median dimensionless linking length b = l_x n^(1/3) / L
and a clustering class measured on a sample of the positions. Any candidate
gives the same labels, so tuning never changes a result, only the time.
"""
from __future__ import annotations

import json
import math
import os
import statistics

import numpy as np

from . import FoF, FoFError, fof_build_cells, fof_finalize, fof_link, schedule_bits

CELL_FACTORS = (0.0, 1.25, 1.375, 1.5, 2.0, 2.5, 3.0, 4.0)
DENSE_MINS = (8, 16, 32)
# one axis at a time, after the grid above; the first value is the default
AXES = {
    "schedule": tuple(schedule_bits(sg, dg, pm) for sg, dg, pm in
                      ((1024, 2048, True), (2048, 2048, True), (512, 2048, True), (1024, 4096, True),
                       (1024, 1024, True), (1024, 2048, False))) + (schedule_bits(giant_skip=True),
                                                                     schedule_bits(tile_join=False)),
    "link_order": ("index", "random"),
    "compression": ("halving", "depth2"),
    "segment_log2": (0, 13, 14, 16),
}
DEFAULTS = {"schedule": 0, "link_order": "index", "compression": "halving", "segment_log2": 0}
DEFAULT_CACHE = os.environ.get("FOF_TUNE_CACHE",
                               os.path.join(os.path.expanduser("~"), ".cache", "paper_2003_11468_amd", "tune.json"))


def clustering_class(pos_host_sample: np.ndarray, box_of_sample: np.ndarray, box: np.ndarray) -> int:
    """log2 of the density-weighted mean overdensity of a sample of positions
    on an 8^3 grid per box: about 0 for uniform points, larger the more the
    particles crowd into halos."""
    if len(pos_host_sample) == 0:
        return 0
    u = pos_host_sample / box[box_of_sample][:, None]
    cell = np.clip((u * 8).astype(np.int64), 0, 7)
    key = box_of_sample * 512 + cell[:, 0] * 64 + cell[:, 1] * 8 + cell[:, 2]
    _, inv, counts = np.unique(key, return_inverse=True, return_counts=True)
    per_box = np.bincount(box_of_sample, minlength=len(box)).astype(np.float64)
    expected = np.maximum(per_box[box_of_sample] / 512.0, 1e-9)
    over = float(np.mean(counts[inv] / expected))
    return int(round(math.log2(max(over, 1.0))))


def workload_key(offsets, box, lx, predicate: str, strict: bool = False, arch: str = "?", clustering: int = 0) -> str:
    off = np.asarray(offsets, dtype=np.int64)
    sizes = np.diff(off)
    n = int(off[-1])
    L = np.broadcast_to(np.asarray(box, dtype=np.float64), sizes.shape)
    l = np.broadcast_to(np.asarray(lx, dtype=np.float64), sizes.shape)
    keep = sizes > 0
    b = float(np.median(l[keep] * np.cbrt(sizes[keep].astype(np.float64)) / L[keep])) if keep.any() else 0.0
    return "%s|%s|%s|n2^%d|boxes2^%d|b%.2g|clu%d" % (predicate, "lt" if strict else "le", arch.split(":")[0],
                                                    round(math.log2(max(n, 1))), round(math.log2(max(len(sizes), 1))),
                                                    b, clustering)


def _sample(pos, offsets, box, k: int = 65536):
    """(positions, box index, box sides) of about k evenly spaced particles."""
    off = np.asarray(offsets, dtype=np.int64)
    n = int(off[-1])
    nb = len(off) - 1
    L = np.ascontiguousarray(np.broadcast_to(np.asarray(box, dtype=np.float64), (nb,)))
    if n == 0:
        return np.zeros((0, 3)), np.zeros(0, dtype=np.int64), L
    step = max(1, n // k)
    idx = np.arange(0, n, step)
    sample = pos[::step].cpu().numpy().astype(np.float64) if hasattr(pos, "cpu") else np.asarray(pos)[idx]
    sample = sample[: len(idx)]
    which = np.searchsorted(off, idx, side="right") - 1
    return sample, which, L


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


def time_config(torch, pos, offsets, box, lx, predicate, strict, cfg: dict, repeats=3, max_workspace=None):
    """Median ms of build+link+finalize for one configuration (None if it cannot run)."""
    kw = {k: cfg[k] for k in ("cell_factor", "dense_min", "schedule", "link_order", "compression") if k in cfg}
    f = FoF(predicate, strict, segment_log2=cfg.get("segment_log2", 0), **kw)
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
             dense_mins=DENSE_MINS, axes: dict | None = None, max_workspace: int | None = None,
             force: bool = False) -> dict:
    """Returns the best configuration for this workload class: cell_factor,
    dense_min, schedule, link_order, compression, segment_log2, and "ms",
    "key", "tried" (every candidate and its time)."""
    import torch

    axes = AXES if axes is None else axes
    arch = torch.cuda.get_device_properties(pos.device).gcnArchName
    clu = clustering_class(*_sample(pos, offsets, box))
    key = workload_key(offsets, box, lx, predicate, strict, arch, clu)
    cache = _load(cache_path) if cache_path else {}
    if not force and key in cache:
        return dict(cache[key], key=key, cached=True)
    if max_workspace is None:
        free, _ = torch.cuda.mem_get_info(pos.device)
        max_workspace = free // 2
    tried = []

    def trial(cfg):
        ms = time_config(torch, pos, offsets, box, lx, predicate, strict, cfg, repeats, max_workspace)
        tried.append(dict(cfg, ms=ms))
        return ms

    best, best_ms = None, None
    for cf in cell_factors:
        for dm in dense_mins:
            cfg = dict(DEFAULTS, cell_factor=cf, dense_min=dm)
            ms = trial(cfg)
            if ms is not None and (best_ms is None or ms < best_ms):
                best, best_ms = cfg, ms
    if best is None:
        raise RuntimeError("no configuration could run")
    for axis, values in axes.items():
        for v in values:
            if v == best.get(axis):
                continue
            cfg = dict(best, **{axis: v})
            ms = trial(cfg)
            if ms is not None and ms < best_ms:
                best, best_ms = cfg, ms
    out = dict(best, ms=best_ms, tried=tried)
    if cache_path:
        cache = _load(cache_path)
        cache[key] = out
        _save(cache_path, cache)
    return dict(out, key=key, cached=False)
