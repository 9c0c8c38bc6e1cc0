"""CPU oracle for periodic Friends-of-Friends labelling (test infrastructure).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg use
this package. It shares no code with the GPU library and the GPU library never
calls it. The arithmetic lives in ``fof_oracle.c`` (plain C, double precision,
no FMA contraction); this file only marshals numpy arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fof_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

STATUS = {0: "ok", -1: "bad particle count", -2: "bad box side", -3: "bad linking length",
          -4: "coordinate outside [0, L) or not finite", -5: "out of host memory"}


class OracleError(RuntimeError):
    pass


def build() -> str:
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
           "-o", _LIB_PATH, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    f32p = ctypes.POINTER(ctypes.c_float)
    i32p = ctypes.POINTER(ctypes.c_int32)
    i64p = ctypes.POINTER(ctypes.c_int64)
    f64p = ctypes.POINTER(ctypes.c_double)
    lib.oracle_r2.argtypes = [f32p, f32p, ctypes.c_double]
    lib.oracle_r2.restype = ctypes.c_double
    for name in ("oracle_fof", "oracle_fof_brute"):
        fn = getattr(lib, name)
        fn.argtypes = [ctypes.c_int64, f32p, ctypes.c_double, ctypes.c_double, ctypes.c_int, i32p, i32p, i64p]
        fn.restype = ctypes.c_int
    lib.oracle_fof_boxes.argtypes = [ctypes.c_int32, i64p, f32p, f64p, f64p, ctypes.c_int, i32p, i32p, i64p,
                                     ctypes.c_int]
    lib.oracle_fof_boxes.restype = ctypes.c_int
    lib.oracle_fof_parallel.argtypes = [ctypes.c_int64, f32p, ctypes.c_double, ctypes.c_double, ctypes.c_int, i32p,
                                        i32p, i64p, ctypes.c_int]
    lib.oracle_fof_parallel.restype = ctypes.c_int
    lib.oracle_cells_per_axis.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_double]
    lib.oracle_cells_per_axis.restype = ctypes.c_int64
    lib.oracle_component.argtypes = [ctypes.c_int64, f32p, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                     ctypes.c_int64, i32p, ctypes.c_int64]
    lib.oracle_component.restype = ctypes.c_int64
    lib.oracle_components_of.argtypes = [ctypes.c_int64, f32p, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                         i64p, ctypes.c_int32, i32p, i64p, i32p]
    lib.oracle_components_of.restype = ctypes.c_int
    _lib = lib
    return lib


def _p(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _pos(pos) -> np.ndarray:
    a = np.ascontiguousarray(pos, dtype=np.float32)
    if a.ndim != 2 or a.shape[1] != 3:
        raise ValueError("positions must be [N, 3] float32")
    return a


def _check(st):
    if st != 0:
        raise OracleError(STATUS.get(st, f"status {st}"))


def r2(a, b, box: float = 1.0) -> float:
    """Canonical squared minimum-image distance of two FP32 points (double)."""
    pa = np.ascontiguousarray(a, dtype=np.float32)
    pb = np.ascontiguousarray(b, dtype=np.float32)
    return float(_load().oracle_r2(_p(pa, ctypes.c_float), _p(pb, ctypes.c_float), box))


def fof(pos, lx: float, box: float = 1.0, strict: bool = False, brute: bool = False):
    """Labels (minimum input index of the group), sizes (at roots) and group count."""
    p = _pos(pos)
    n = len(p)
    label = np.empty(n, dtype=np.int32)
    size = np.empty(n, dtype=np.int32)
    ng = ctypes.c_int64(0)
    fn = _load().oracle_fof_brute if brute else _load().oracle_fof
    _check(fn(n, _p(p, ctypes.c_float), float(box), float(lx), int(strict), _p(label, ctypes.c_int32),
              _p(size, ctypes.c_int32), ctypes.byref(ng)))
    return label, size, int(ng.value)


def fof_parallel(pos, lx: float, box: float = 1.0, strict: bool = False, threads: int = 1):
    """The same outputs as fof(), with the link search over host threads (for
    inputs of up to ~10^9 particles)."""
    p = _pos(pos)
    n = len(p)
    label = np.empty(n, dtype=np.int32)
    size = np.empty(n, dtype=np.int32)
    ng = ctypes.c_int64(0)
    _check(_load().oracle_fof_parallel(n, _p(p, ctypes.c_float), float(box), float(lx), int(strict),
                                       _p(label, ctypes.c_int32), _p(size, ctypes.c_int32), ctypes.byref(ng),
                                       int(threads)))
    return label, size, int(ng.value)


def fof_boxes(pos, offsets, box, lx, strict: bool = False, threads: int = 1):
    """Independent boxes; labels are box-local indices."""
    p = _pos(pos)
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    L = np.ascontiguousarray(box, dtype=np.float64)
    l = np.ascontiguousarray(lx, dtype=np.float64)
    nb = len(L)
    if len(off) != nb + 1 or len(l) != nb or off[-1] != len(p):
        raise ValueError("inconsistent box description")
    label = np.empty(len(p), dtype=np.int32)
    size = np.empty(len(p), dtype=np.int32)
    ng = np.zeros(nb, dtype=np.int64)
    _check(_load().oracle_fof_boxes(nb, _p(off, ctypes.c_int64), _p(p, ctypes.c_float), _p(L, ctypes.c_double),
                                    _p(l, ctypes.c_double), int(strict), _p(label, ctypes.c_int32),
                                    _p(size, ctypes.c_int32), _p(ng, ctypes.c_int64), int(threads)))
    return label, size, ng


def cells_per_axis(n: int, lx: float, box: float = 1.0) -> int:
    return int(_load().oracle_cells_per_axis(n, box, lx))


def component(pos, lx: float, start: int, box: float = 1.0, strict: bool = False) -> np.ndarray:
    """Sorted members of the group containing particle `start` (breadth-first search)."""
    p = _pos(pos)
    cap = 1 << 16
    while True:
        out = np.empty(cap, dtype=np.int32)
        c = _load().oracle_component(len(p), _p(p, ctypes.c_float), float(box), float(lx), int(strict),
                                     int(start), _p(out, ctypes.c_int32), cap)
        if c < 0:
            _check(int(c))
        if c <= cap:
            return out[:c].copy()
        cap = int(c)


def components_of(pos, lx: float, starts, box: float = 1.0, strict: bool = False):
    """Groups of several start particles by breadth-first search over one cell
    list: (sizes[k], minimum index[k], mark) with mark[i] = k for the members
    found from start k (-1 elsewhere; a start inside an earlier start's group
    gets that group's size and minimum and marks nothing)."""
    p = _pos(pos)
    st = np.ascontiguousarray(starts, dtype=np.int64)
    mark = np.empty(len(p), dtype=np.int32)
    sizes = np.zeros(len(st), dtype=np.int64)
    mins = np.zeros(len(st), dtype=np.int32)
    _check(_load().oracle_components_of(len(p), _p(p, ctypes.c_float), float(box), float(lx), int(strict),
                                        _p(st, ctypes.c_int64), len(st), _p(mark, ctypes.c_int32),
                                        _p(sizes, ctypes.c_int64), _p(mins, ctypes.c_int32)))
    return sizes, mins, mark
