"""Periodic Friends-of-Friends labelling on an AMD Instinct MI355X (gfx950).

Thin ctypes binding of the C-ABI in ``include/fof.h``; every step of the
labelling runs in the HIP kernels of ``libfof_gfx950.so``. PyTorch only
provides device memory and the stream. There is no CPU fallback: without the
built library every entry point raises.

Low-level functions carry the C names (``fof_create``, ``fof_build_cells``,
``fof_link``, ``fof_finalize``, ...). ``FoF`` and ``label`` wrap them for
tensors::

    label, size, n_groups = paper_2003_11468_amd.label(pos_cuda_f32_nx3, lx=0.2/256)
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfof_gfx950.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "fof.h")

FOF_OK, FOF_ERR_INVALID_ARG, FOF_ERR_OUT_OF_BOX, FOF_ERR_BAD_STATE, FOF_ERR_WORKSPACE, FOF_ERR_DEVICE, \
    FOF_ERR_UNSUPPORTED = range(7)
FOF_PRED_FP64, FOF_PRED_FP32_FILTER = 0, 1
PREDICATES = {"fp64": FOF_PRED_FP64, "fp32_filter": FOF_PRED_FP32_FILTER}
LINK_ORDERS = {"index": 0, "random": 1}   # fof_options.link_order


class FoFError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = _lib.fof_status_string(status).decode() if _lib is not None else str(status)
        super().__init__(f"{where}: {msg} (status {status})")


class Options(ctypes.Structure):
    _fields_ = [("predicate", ctypes.c_int32), ("strict_less", ctypes.c_int32), ("cell_factor", ctypes.c_double),
                ("collect_stats", ctypes.c_int32), ("dense_min", ctypes.c_int32), ("collect_timings", ctypes.c_int32),
                ("sort_segment_log2", ctypes.c_int32), ("domains", ctypes.c_int32),
                ("link_order", ctypes.c_int32), ("schedule", ctypes.c_int32), ("compression", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 2)]


class Stats(ctypes.Structure):
    _fields_ = [("n_particles", ctypes.c_int64), ("n_cells", ctypes.c_int64), ("n_groups", ctypes.c_int64),
                ("pair_tests", ctypes.c_int64), ("links", ctypes.c_int64), ("band_hits", ctypes.c_int64),
                ("cas_retries", ctypes.c_int64), ("fp64_boxes", ctypes.c_int64),
                ("sparse_pair_tests", ctypes.c_int64), ("queued_links", ctypes.c_int64),
                ("dense_items", ctypes.c_int64), ("boundary_links", ctypes.c_int64),
                ("boundary_groups", ctypes.c_int64), ("find_depth_max", ctypes.c_int64),
                ("find_depth_sum", ctypes.c_int64), ("reserved", ctypes.c_int64 * 1)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class BoxInfo(ctypes.Structure):
    _fields_ = [("cells_per_axis", ctypes.c_int64), ("l2", ctypes.c_double), ("lo32", ctypes.c_float),
                ("hi32", ctypes.c_float), ("fp64_only", ctypes.c_int32), ("sub_cells_per_axis", ctypes.c_int32),
                ("sub_cells_adjacent", ctypes.c_int32), ("reserved", ctypes.c_int32 * 1)]


_lib = None
EXPORTS = ["fof_default_options", "fof_create", "fof_set_stream", "fof_workspace_bytes", "fof_set_workspace",
           "fof_build_cells", "fof_link", "fof_finalize", "fof_read_n_groups", "fof_get_stats",
           "fof_graph_capture", "fof_graph_launch", "fof_destroy", "fof_status_string", "fof_get_kernel_times",
           "fof_kernel_name", "fof_describe_box", "fof_catalogue", "fof_relink", "fof_label_noalloc"]
NOALLOC_SCRATCH_BYTES = 128 << 20   # FOF_NOALLOC_SCRATCH_BYTES


def load_library():
    """Load the built library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run paper_2003_11468_amd/build.py (hipcc, gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    i64p, f64p = ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_double)
    sig = {
        "fof_default_options": (None, [ctypes.POINTER(Options)]),
        "fof_create": (ctypes.c_int, [ctypes.POINTER(vp), ctypes.POINTER(Options), vp]),
        "fof_set_stream": (ctypes.c_int, [vp, vp]),
        "fof_workspace_bytes": (ctypes.c_int, [vp, i64p, f64p, f64p, i32, ctypes.POINTER(sz)]),
        "fof_set_workspace": (ctypes.c_int, [vp, vp, sz]),
        "fof_build_cells": (ctypes.c_int, [vp, vp, i64p, f64p, f64p, i32]),
        "fof_link": (ctypes.c_int, [vp]),
        "fof_finalize": (ctypes.c_int, [vp, vp, vp, i64p]),
        "fof_read_n_groups": (ctypes.c_int, [vp, i64p]),
        "fof_get_stats": (ctypes.c_int, [vp, ctypes.POINTER(Stats)]),
        "fof_graph_capture": (ctypes.c_int, [vp, vp, i64p, f64p, f64p, i32, vp, vp]),
        "fof_graph_launch": (ctypes.c_int, [vp]),
        "fof_destroy": (ctypes.c_int, [vp]),
        "fof_status_string": (ctypes.c_char_p, [ctypes.c_int]),
        "fof_get_kernel_times": (ctypes.c_int, [vp, f64p, ctypes.POINTER(i32), i32, ctypes.POINTER(i32)]),
        "fof_kernel_name": (ctypes.c_char_p, [i32]),
        "fof_describe_box": (ctypes.c_int, [ctypes.POINTER(Options), i64, ctypes.c_double, ctypes.c_double,
                                            ctypes.POINTER(BoxInfo)]),
        "fof_catalogue": (ctypes.c_int, [vp, vp, vp, i32, vp, vp, vp, i64, i64p]),
        "fof_relink": (ctypes.c_int, [vp, f64p, i32]),
        "fof_label_noalloc": (ctypes.c_int, [ctypes.POINTER(Options), vp, vp, i64, ctypes.c_double, ctypes.c_double,
                                             vp, vp, i64p]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(st: int, where: str):
    if st != FOF_OK:
        raise FoFError(st, where)


def _arr(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _p(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _boxes(offsets, box, lx):
    off = _arr(offsets, np.int64)
    L = _arr(np.broadcast_to(np.asarray(box, dtype=np.float64), (len(off) - 1,)), np.float64)
    l = _arr(np.broadcast_to(np.asarray(lx, dtype=np.float64), (len(off) - 1,)), np.float64)
    return off, L, l


def _dptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


# ------------------------------------------------------------- C names --

def fof_default_options() -> Options:
    o = Options()
    load_library().fof_default_options(ctypes.byref(o))
    return o


def fof_create(opt: Options | None = None, stream: int | None = None) -> ctypes.c_void_p:
    ctx = ctypes.c_void_p()
    _check(load_library().fof_create(ctypes.byref(ctx), ctypes.byref(opt) if opt is not None else None,
                                     ctypes.c_void_p(stream or 0)), "fof_create")
    return ctx


def fof_set_stream(ctx, stream: int):
    _check(load_library().fof_set_stream(ctx, ctypes.c_void_p(stream)), "fof_set_stream")


def fof_workspace_bytes(ctx, offsets, box, lx) -> int:
    off, L, l = _boxes(offsets, box, lx)
    out = ctypes.c_size_t()
    _check(load_library().fof_workspace_bytes(ctx, _p(off, ctypes.c_int64), _p(L, ctypes.c_double),
                                              _p(l, ctypes.c_double), len(L), ctypes.byref(out)),
           "fof_workspace_bytes")
    return int(out.value)


def fof_set_workspace(ctx, ws, nbytes: int | None = None):
    ptr = _dptr(ws)
    n = nbytes if nbytes is not None else (ws.numel() * ws.element_size() if ws is not None else 0)
    _check(load_library().fof_set_workspace(ctx, ctypes.c_void_p(ptr), n), "fof_set_workspace")


def fof_build_cells(ctx, pos, offsets, box, lx):
    off, L, l = _boxes(offsets, box, lx)
    _check(load_library().fof_build_cells(ctx, ctypes.c_void_p(_dptr(pos)), _p(off, ctypes.c_int64),
                                          _p(L, ctypes.c_double), _p(l, ctypes.c_double), len(L)),
           "fof_build_cells")


def fof_link(ctx):
    _check(load_library().fof_link(ctx), "fof_link")


def fof_finalize(ctx, group_index, group_size, n_boxes: int | None = None):
    """With n_boxes, waits and returns the per-box group counts."""
    out = None
    ptr = None
    if n_boxes is not None:
        out = np.zeros(n_boxes, dtype=np.int64)
        ptr = _p(out, ctypes.c_int64)
    _check(load_library().fof_finalize(ctx, ctypes.c_void_p(_dptr(group_index)),
                                       ctypes.c_void_p(_dptr(group_size)), ptr), "fof_finalize")
    return out


def fof_read_n_groups(ctx, n_boxes: int) -> np.ndarray:
    out = np.zeros(n_boxes, dtype=np.int64)
    _check(load_library().fof_read_n_groups(ctx, _p(out, ctypes.c_int64)), "fof_read_n_groups")
    return out


def fof_get_stats(ctx) -> dict:
    s = Stats()
    _check(load_library().fof_get_stats(ctx, ctypes.byref(s)), "fof_get_stats")
    return s.as_dict()


def fof_graph_capture(ctx, pos, offsets, box, lx, group_index, group_size):
    off, L, l = _boxes(offsets, box, lx)
    _check(load_library().fof_graph_capture(ctx, ctypes.c_void_p(_dptr(pos)), _p(off, ctypes.c_int64),
                                            _p(L, ctypes.c_double), _p(l, ctypes.c_double), len(L),
                                            ctypes.c_void_p(_dptr(group_index)),
                                            ctypes.c_void_p(_dptr(group_size))), "fof_graph_capture")


def fof_graph_launch(ctx):
    _check(load_library().fof_graph_launch(ctx), "fof_graph_launch")


def fof_destroy(ctx):
    if ctx is not None and ctx.value:
        _check(load_library().fof_destroy(ctx), "fof_destroy")


def fof_get_kernel_times(ctx) -> dict:
    """{kernel name: (ms summed, launches)} since the previous call."""
    cap = 32
    ms = np.zeros(cap, dtype=np.float64)
    cnt = np.zeros(cap, dtype=np.int32)
    nk = ctypes.c_int32()
    _check(load_library().fof_get_kernel_times(ctx, _p(ms, ctypes.c_double), _p(cnt, ctypes.c_int32), cap,
                                               ctypes.byref(nk)), "fof_get_kernel_times")
    lib = load_library()
    return {lib.fof_kernel_name(k).decode(): (float(ms[k]), int(cnt[k])) for k in range(nk.value)}


def fof_describe_box(n_particles: int, box: float, lx: float, opt: Options | None = None) -> dict:
    """Host only: cells per axis and the FP32 decision thresholds for one box."""
    info = BoxInfo()
    _check(load_library().fof_describe_box(ctypes.byref(opt) if opt is not None else None, int(n_particles),
                                           float(box), float(lx), ctypes.byref(info)), "fof_describe_box")
    return {k: getattr(info, k) for k, _ in info._fields_ if k != "reserved"}


def fof_catalogue(ctx, label, size, min_size: int, first=None, gsize=None, gbox=None, capacity: int = 0) -> int:
    """Groups of at least min_size members (see include/fof.h); returns how many there are."""
    count = ctypes.c_int64(0)
    _check(load_library().fof_catalogue(ctx, _dptr(label), _dptr(size), int(min_size), _dptr(first), _dptr(gsize),
                                        _dptr(gbox), int(capacity), ctypes.byref(count)), "fof_catalogue")
    return int(count.value)


def fof_relink(ctx, lx, n_boxes: int):
    """New linking lengths (one per box, each at most the build's) over the built cells."""
    l = _arr(np.broadcast_to(np.asarray(lx, dtype=np.float64), (int(n_boxes),)), np.float64)
    _check(load_library().fof_relink(ctx, l.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(n_boxes)),
           "fof_relink")


def fof_label_noalloc(pos, box, lx, group_index, group_size, opt: Options | None = None, stream: int | None = None,
                      sync: bool = True):
    """One box through the library's own device scratch (no workspace, no
    allocation; see include/fof.h). Returns the group count when sync."""
    ng = ctypes.c_int64(0)
    n = 0 if pos is None else int(pos.shape[0])
    _check(load_library().fof_label_noalloc(ctypes.byref(opt) if opt is not None else None,
                                            ctypes.c_void_p(stream or 0), ctypes.c_void_p(_dptr(pos)), n,
                                            float(box), float(lx), ctypes.c_void_p(_dptr(group_index)),
                                            ctypes.c_void_p(_dptr(group_size)),
                                            ctypes.byref(ng) if sync else None), "fof_label_noalloc")
    return int(ng.value) if sync else None


def fof_kernel_name(k: int) -> str:
    return load_library().fof_kernel_name(k).decode()


def fof_status_string(status: int) -> str:
    return load_library().fof_status_string(status).decode()


# ------------------------------------------------------ tensor wrapper --

COMPRESSIONS = {"halving": 0, "depth2": 1}   # fof_options.compression


def schedule_bits(sparse_grid: int = 1024, dense_grid: int = 2048, premerge: bool = True,
                  giant_skip: bool = False, tile_join: bool = True) -> int:
    """fof_options.schedule from its parts (grids of the two persistent link kernels, pre-merge,
    giant-component skip, links inside a tile joined by the search)."""
    sg = {1024: 0, 512: 1, 2048: 2, 4096: 3}[int(sparse_grid)]
    dg = {2048: 0, 1024: 1, 4096: 2, 8192: 3}[int(dense_grid)]
    return sg | (dg << 2) | (0 if premerge else 16) | (32 if giant_skip else 0) | (0 if tile_join else 64)


def make_options(predicate: str = "fp32_filter", strict: bool = False, cell_factor: float = 0.0,
                 stats: bool = False, dense_min: int = 0, timings: bool = False, segment_log2: int = 0,
                 domains: int = 0, link_order: str = "index", schedule: int = 0,
                 compression: str = "halving") -> Options:
    o = fof_default_options()
    o.schedule = int(schedule)
    o.compression = COMPRESSIONS[compression]
    o.sort_segment_log2 = int(segment_log2)
    o.domains = int(domains)
    o.link_order = LINK_ORDERS[link_order]
    o.collect_timings = int(timings)
    o.predicate = PREDICATES[predicate]
    o.strict_less = int(strict)
    o.cell_factor = float(cell_factor)
    o.collect_stats = int(stats)
    o.dense_min = int(dense_min)
    return o


class FoF:
    """A context plus a workspace tensor, reused across calls of the same shape."""

    def __init__(self, predicate: str = "fp32_filter", strict: bool = False, cell_factor: float = 0.0,
                 stats: bool = False, stream=None, dense_min: int = 0, timings: bool = False,
                 segment_log2: int = 0, domains: int = 0, link_order: str = "index", schedule: int = 0,
                 compression: str = "halving"):
        import torch

        self._torch = torch
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.ctx = fof_create(make_options(predicate, strict, cell_factor, stats, dense_min, timings, segment_log2,
                                           domains, link_order, schedule, compression), self.stream.cuda_stream)
        self.ws = None
        self._graph_refs = None   # tensors a captured graph reads or writes

    def close(self):
        if self.ctx is not None:
            fof_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def reserve(self, offsets, box, lx):
        need = fof_workspace_bytes(self.ctx, offsets, box, lx)
        if self.ws is None or self.ws.numel() < need:
            self.ws = self._torch.empty(max(need, 256), dtype=self._torch.uint8, device=self.stream.device)
            fof_set_workspace(self.ctx, self.ws)   # discards a captured graph
            self._graph_refs = None
        return need

    def outputs(self, n: int):
        t = self._torch
        return (t.empty(n, dtype=t.int32, device=self.stream.device),
                t.empty(n, dtype=t.int32, device=self.stream.device))

    def run(self, pos, offsets, box, lx, label=None, size=None, sync: bool = True):
        """build + link + finalize. Returns (label, size, n_groups or None)."""
        self._check_pos(pos, offsets)
        self.reserve(offsets, box, lx)
        if label is None or size is None:
            label, size = self.outputs(pos.shape[0])
        self._n = pos.shape[0]
        fof_build_cells(self.ctx, pos, offsets, box, lx)
        fof_link(self.ctx)
        ng = fof_finalize(self.ctx, label, size, len(offsets) - 1 if sync else None)
        return label, size, ng

    def capture(self, pos, offsets, box, lx, label, size):
        self._check_pos(pos, offsets)
        self.reserve(offsets, box, lx)
        fof_graph_capture(self.ctx, pos, offsets, box, lx, label, size)
        # the graph holds raw pointers: keep its tensors alive with it
        self._graph_refs = (pos, label, size, self.ws)

    def replay(self):
        fof_graph_launch(self.ctx)

    def n_groups(self, n_boxes: int) -> np.ndarray:
        return fof_read_n_groups(self.ctx, n_boxes)

    def stats(self) -> dict:
        return fof_get_stats(self.ctx)

    def kernel_times(self) -> dict:
        return fof_get_kernel_times(self.ctx)

    def relink(self, lx, n_boxes: int, label=None, size=None, sync: bool = True):
        """Groups at new linking lengths (each at most the last build's) over the cells of the
        last run. Returns (label, size, n_groups or None) like run()."""
        if label is None or size is None:
            label, size = self.outputs(int(self._n))
        fof_relink(self.ctx, lx, n_boxes)
        fof_link(self.ctx)
        ng = fof_finalize(self.ctx, label, size, n_boxes if sync else None)
        return label, size, ng

    def catalogue(self, label, size, min_size: int = 1):
        """(first, size, box) tensors of the groups of at least min_size members of the
        last run's outputs, in order of box and label."""
        t = self._torch
        n = fof_catalogue(self.ctx, label, size, min_size)
        dev = self.stream.device
        first, gsize, gbox = (t.empty(max(n, 1), dtype=t.int32, device=dev) for _ in range(3))
        got = fof_catalogue(self.ctx, label, size, min_size, first, gsize, gbox, n)
        assert got == n
        return first[:n], gsize[:n], gbox[:n]

    def _check_pos(self, pos, offsets):
        t = self._torch
        if not (pos.is_cuda and pos.dtype == t.float32 and pos.dim() == 2 and pos.shape[1] == 3
                and pos.is_contiguous()):
            raise ValueError("positions must be a contiguous [N, 3] float32 tensor on the GPU")
        if int(np.asarray(offsets)[-1]) != pos.shape[0]:
            raise ValueError("box offsets do not cover the position array")


def label(pos, lx, box: float = 1.0, predicate: str = "fp32_filter", strict: bool = False,
          cell_factor: float = 0.0, dense_min: int = 0):
    """Single periodic box: (group_index, group_size, n_groups)."""
    f = FoF(predicate, strict, cell_factor, dense_min=dense_min)
    try:
        lab, size, ng = f.run(pos, [0, pos.shape[0]], box, lx)
        return lab, size, int(ng[0])
    finally:
        f.close()


def label_boxes(pos, offsets, box, lx, predicate: str = "fp32_filter", strict: bool = False,
                cell_factor: float = 0.0, dense_min: int = 0):
    """Many independent boxes in one pass; labels are box-local."""
    f = FoF(predicate, strict, cell_factor, dense_min=dense_min)
    try:
        return f.run(pos, offsets, box, lx)
    finally:
        f.close()
