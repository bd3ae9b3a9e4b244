"""Seeded observer (candidate transmitter) lists.

Observers are {x (column), y (row), roi, h_t, h_r} int32 records.  These are
inputs only: the uneven-batch workload draws its candidates uniformly over
the terrain with a per-candidate ROI and height, and forces the four corners
and four edge midpoints so that clipped windows are always exercised.
"""
from __future__ import annotations

import numpy as np

OBSERVER_DTYPE = np.dtype([("x", "<i4"), ("y", "<i4"), ("roi", "<i4"),
                           ("h_t", "<i4"), ("h_r", "<i4")])


def uniform_observers(nrows: int, ncols: int, n: int, seed: int, roi=(50, 400),
                      height=(5, 100), force_edges: bool = True) -> np.ndarray:
    """n distinct posts (the 8 edge posts first when force_edges), ROI drawn
    uniformly from the integer range roi=(lo, hi) and a height from
    height=(lo, hi) used for both h_t and h_r."""
    rng = np.random.Generator(np.random.PCG64(seed))
    forced = []
    if force_edges:
        forced = [(0, 0), (ncols - 1, 0), (0, nrows - 1), (ncols - 1, nrows - 1),
                  (ncols // 2, 0), (ncols // 2, nrows - 1), (0, nrows // 2), (ncols - 1, nrows // 2)]
    seen = set()
    xs, ys = [], []
    for (x, y) in forced:
        if (x, y) not in seen and len(xs) < n:
            seen.add((x, y)); xs.append(x); ys.append(y)
    while len(xs) < n:
        need = n - len(xs)
        lin = rng.integers(0, nrows * ncols, size=2 * need + 16)
        for v in lin.tolist():
            y, x = divmod(v, ncols)
            if (x, y) in seen:
                continue
            seen.add((x, y)); xs.append(x); ys.append(y)
            if len(xs) == n:
                break
    o = np.zeros(n, OBSERVER_DTYPE)
    o["x"] = xs
    o["y"] = ys
    o["roi"] = rng.integers(roi[0], roi[1] + 1, size=n)
    h = rng.integers(height[0], height[1] + 1, size=n)
    o["h_t"] = h
    o["h_r"] = h
    return o


def grid_observers(cand: np.ndarray, ncols: int, roi: int, h_t: int, h_r: int) -> np.ndarray:
    """Observer records for candidate linear post indices (-1 entries are
    dropped), all sharing one ROI and height pair."""
    cand = np.asarray(cand, np.int64)
    cand = cand[cand >= 0]
    o = np.zeros(cand.shape[0], OBSERVER_DTYPE)
    o["y"] = cand // ncols
    o["x"] = cand % ncols
    o["roi"] = roi
    o["h_t"] = h_t
    o["h_r"] = h_r
    return o
