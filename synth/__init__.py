"""Seeded synthetic inputs shaped like N-body snapshots (inputs only).

Both the GPU path and the CPU oracle are fed from this module; it holds none
of the Friends-of-Friends arithmetic. The C core (``synth.c``) is a
counter-based generator (Philox4x32-10), so every workload is reproducible
bit for bit from its seed.

Workloads (box side L = 1, linking length l_x = b x mean separation):

``uniform32k``     N = 32^3 i.i.d. uniform, b = 0.2, seed 0.
``clustered256``   N = 256^3, 60 % of particles in Plummer halos with counts
                   from dN/dM ~ M^-1.9 on [20, 1e5], 40 % uniform, b = 0.2, seed 1.
``clustered512``   N = 512^3, same generator with 70 % in halos, b = 0.2, seed 2.
``batched256``     256 independent boxes, N_b = round(exp(U[ln 1e3, ln 1e6])),
                   each from the clustered256 generator (60 % halos), its own
                   l_x = 0.2 / cbrt(N_b); seed 3, box b uses stream b.
``percolate1024``  N = 1024^3, 90 % in halos, counts on [20, 1e6], b = 0.5, seed 4.
                   Its largest group holds about 1e4 particles: it does not percolate.
``lattice1024``    N = 1024^3 on a cubic lattice of spacing s = 0.9 l_x, each site
                   jittered by up to 2 % of s per axis, seed 5: every particle links
                   exactly its six axis neighbours (at most 1.042 s < l_x = 1.111 s
                   apart; diagonal neighbours stay at least 1.357 s apart), so the
                   whole box is one group of 1024^3, the most contended input for
                   the union-find.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_LIB_PATH = os.path.join(_HERE, "libsynth.so")
_lib = None


def build() -> str:
    """Compile the generator (gcc, OpenMP)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", _LIB_PATH, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    f32p = ctypes.POINTER(ctypes.c_float)
    i64p = ctypes.POINTER(ctypes.c_int64)
    lib.synth_philox4x32_10.argtypes = [u32p, u32p, u32p]
    lib.synth_philox4x32_10.restype = None
    lib.synth_permute.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64]
    lib.synth_permute.restype = ctypes.c_uint64
    lib.synth_uniform.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_uint32, ctypes.c_uint32, f32p]
    lib.synth_uniform.restype = None
    lib.synth_halo_counts.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_uint32, ctypes.c_uint32, i64p, ctypes.c_int64]
    lib.synth_halo_counts.restype = ctypes.c_int64
    lib.synth_clustered.argtypes = [ctypes.c_int64, ctypes.c_double, i64p, ctypes.c_int64,
                                    ctypes.c_uint32, ctypes.c_uint32, f32p]
    lib.synth_clustered.restype = None
    lib.synth_lattice.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_double, ctypes.c_uint32,
                                  ctypes.c_uint32, f32p]
    lib.synth_lattice.restype = None
    lib.synth_box_sizes.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_uint32, i64p]
    lib.synth_box_sizes.restype = None
    _lib = lib
    return lib


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def philox4x32_10(ctr, key) -> np.ndarray:
    lib = _load()
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib.synth_philox4x32_10(_ptr(c, ctypes.c_uint32), _ptr(k, ctypes.c_uint32), _ptr(out, ctypes.c_uint32))
    return out


def permute(n: int, seed: int, stream: int, k: int) -> int:
    return int(_load().synth_permute(n, seed, stream, k))


def uniform(n: int, seed: int, stream: int = 0, box: float = 1.0) -> np.ndarray:
    pos = np.empty((n, 3), dtype=np.float32)
    if n:
        _load().synth_uniform(n, box, seed, stream, _ptr(pos, ctypes.c_float))
    return pos


def halo_counts(budget: int, m_min: float, m_max: float, slope: float, seed: int, stream: int = 0) -> np.ndarray:
    cap = max(16, int(budget // max(1.0, m_min * 0.5)) + 16)
    counts = np.empty(cap, dtype=np.int64)
    h = _load().synth_halo_counts(budget, m_min, m_max, slope, seed, stream, _ptr(counts, ctypes.c_int64), cap)
    if h < 0:
        raise RuntimeError("halo table overflow")
    return counts[:h].copy()


def clustered(n: int, seed: int, stream: int = 0, halo_frac: float = 0.6, m_min: float = 20.0,
              m_max: float = 1e5, slope: float = 1.9, box: float = 1.0) -> np.ndarray:
    budget = int(round(halo_frac * n))
    counts = halo_counts(budget, m_min, m_max, slope, seed, stream)
    pos = np.empty((n, 3), dtype=np.float32)
    if n:
        _load().synth_clustered(n, box, _ptr(counts, ctypes.c_int64), len(counts), seed, stream,
                                _ptr(pos, ctypes.c_float))
    return pos


def jittered_lattice(side: int, jitter: float, seed: int, stream: int = 0, box: float = 1.0) -> np.ndarray:
    """side^3 lattice sites of spacing box/side, each coordinate moved by a
    uniform offset of up to `jitter` spacings, in shuffled order."""
    pos = np.empty((side ** 3, 3), dtype=np.float32)
    if side:
        _load().synth_lattice(side, box, jitter, seed, stream, _ptr(pos, ctypes.c_float))
    return pos


def box_sizes(n_boxes: int, lo: float, hi: float, seed: int) -> np.ndarray:
    out = np.empty(n_boxes, dtype=np.int64)
    _load().synth_box_sizes(n_boxes, lo, hi, seed, _ptr(out, ctypes.c_int64))
    return out


def linking_length(b: float, n: int, box: float = 1.0) -> float:
    """l_x = b * L / n^(1/3), with the integer cube root used when n is a cube."""
    side = round(n ** (1.0 / 3.0))
    root = float(side) if side ** 3 == n else float(np.cbrt(float(n)))
    return b * box / root


@dataclass
class Workload:
    """Concatenated boxes: box k holds particles offsets[k]:offsets[k+1]."""
    name: str
    pos: np.ndarray            # float32 [N_total, 3]
    offsets: np.ndarray        # int64 [n_boxes + 1]
    box: np.ndarray            # float64 [n_boxes]
    lx: np.ndarray             # float64 [n_boxes]
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.offsets[-1])

    @property
    def n_boxes(self) -> int:
        return len(self.box)


def _single(name, pos, b, meta):
    n = len(pos)
    return Workload(name, pos, np.array([0, n], dtype=np.int64), np.array([1.0]),
                    np.array([linking_length(b, n)]), dict(meta, b=b))


RECIPES = {
    "uniform32k": dict(kind="uniform", n=32 ** 3, b=0.2, seed=0),
    "clustered256": dict(kind="clustered", n=256 ** 3, b=0.2, seed=1, halo_frac=0.6, m_max=1e5),
    "clustered512": dict(kind="clustered", n=512 ** 3, b=0.2, seed=2, halo_frac=0.7, m_max=1e5),
    "batched256": dict(kind="batched", n_boxes=256, lo=1e3, hi=1e6, b=0.2, seed=3, halo_frac=0.6, m_max=1e5),
    "percolate1024": dict(kind="clustered", n=1024 ** 3, b=0.5, seed=4, halo_frac=0.9, m_max=1e6),
    "lattice1024": dict(kind="lattice", side=1024, spacing_over_lx=0.9, jitter=0.02, seed=5),
}


def make(name: str, n: int | None = None, n_boxes: int | None = None, size_scale: float = 1.0) -> Workload:
    """Build a named workload; `n` / `n_boxes` / `size_scale` shrink it for tests."""
    r = dict(RECIPES[name])
    if r["kind"] == "uniform":
        n = r["n"] if n is None else n
        return _single(name, uniform(n, r["seed"]), r["b"], dict(r, n=n))
    if r["kind"] == "clustered":
        n = r["n"] if n is None else n
        pos = clustered(n, r["seed"], 0, r["halo_frac"], 20.0, r["m_max"], 1.9)
        return _single(name, pos, r["b"], dict(r, n=n))
    if r["kind"] == "lattice":
        side = r["side"] if n is None else int(round(n ** (1.0 / 3.0)))
        pos = jittered_lattice(side, r["jitter"], r["seed"])
        lx = (1.0 / side) / r["spacing_over_lx"]
        return Workload(name, pos, np.array([0, side ** 3], dtype=np.int64), np.array([1.0]), np.array([lx]),
                        dict(r, side=side))
    nb = r["n_boxes"] if n_boxes is None else n_boxes
    sizes = box_sizes(nb, r["lo"], r["hi"], r["seed"])
    sizes = np.maximum(1, np.round(sizes * size_scale)).astype(np.int64)
    offsets = np.zeros(nb + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)
    pos = np.empty((int(offsets[-1]), 3), dtype=np.float32)
    lx = np.empty(nb)
    for k in range(nb):
        nk = int(sizes[k])
        pos[offsets[k]:offsets[k + 1]] = clustered(nk, r["seed"], k, r["halo_frac"], 20.0, r["m_max"], 1.9)
        lx[k] = linking_length(r["b"], nk)
    return Workload(name, pos, offsets, np.ones(nb), lx, dict(r, n_boxes=nb, size_scale=size_scale))
