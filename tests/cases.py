"""Hand-built inputs shared by the oracle pins and the GPU parity tests.

Only inputs and expected values derived by hand live here; nothing in this
file computes a link, a distance or a component.
"""
from __future__ import annotations

import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_fixture(name: str) -> dict:
    out = {"pos": []}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, *vals = line.split()
            if key == "L_LX":
                out["box"], out["lx"] = float(vals[0]), float(vals[1])
            elif key == "P":
                out["pos"].append([float(v) for v in vals])
            else:
                out[key.lower()] = np.array([int(v) for v in vals], dtype=np.int64)
    out["pos"] = np.array(out["pos"], dtype=np.float32)
    return out


def lattice(n: int, box: float = 1.0, seed: int = 0) -> np.ndarray:
    """Simple cubic lattice with spacing box/n, shuffled (seeded)."""
    g = (np.arange(n, dtype=np.float64) * (box / n)).astype(np.float32)
    x, y, z = np.meshgrid(g, g, g, indexing="ij")
    pos = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(pos[rng.permutation(len(pos))])


def chain_across_boundary(n: int, step: float, axis: int, y0: float = 0.5) -> np.ndarray:
    """n points spaced `step` along `axis`, centred on the periodic face 0 / L."""
    pos = np.full((n, 3), y0, dtype=np.float64)
    t = (np.arange(n) - n // 2) * step
    pos[:, axis] = np.mod(t, 1.0)
    return pos.astype(np.float32)


def labels_from_partition(groups: list[list[int]], n: int) -> tuple[np.ndarray, np.ndarray]:
    """Canonical labels (group minimum) and root sizes for an explicit partition."""
    label = np.arange(n, dtype=np.int64)
    size = np.zeros(n, dtype=np.int64)
    seen = np.zeros(n, dtype=bool)
    for g in groups:
        m = min(g)
        for i in g:
            label[i] = m
            seen[i] = True
        size[m] = len(g)
    for i in range(n):
        if not seen[i]:
            size[i] = 1
    return label, size
