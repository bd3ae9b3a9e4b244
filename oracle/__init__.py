"""CPU oracle for the multiple-observer siting method (arXiv 2006.16783).

TEST INFRASTRUCTURE ONLY: the test-suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package; the product path
(the HIP library and its Python binding) never does, and shares no code with
it.  The arithmetic lives in ``oracle.c`` (plain C, exact integers) and, for
the learned ranking, in ``cnn.py`` (numpy, float64).  This module only loads
the compiled C file and marshals numpy arrays into it.

Every function states the passage of the paper it follows; the C source holds
the step-by-step definitions.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

OBSERVER_DTYPE = np.dtype([("x", "<i4"), ("y", "<i4"), ("roi", "<i4"),
                           ("h_t", "<i4"), ("h_r", "<i4")])


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (OpenMP over independent posts/observers)."""
    if force or not os.path.exists(_LIB_PATH) or \
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        build()
        lib = C.CDLL(_LIB_PATH)
        P = C.c_void_p
        i64, i32, u64 = C.c_int64, C.c_int32, C.c_uint64
        lib.or_philox4x32_10.argtypes = [P, P, P]
        lib.or_los.argtypes = [P, i64, i64, i64, i64, i64, i64, i64, i32, i32]
        lib.or_los.restype = C.c_int
        lib.or_vix.argtypes = [P, i64, i64, i64, i32, i32, i32, i32, u64, P, i64, i64]
        lib.or_vix_rowlist.argtypes = [P, i64, i64, i64, i32, i32, i32, i32, u64, P, i64, P]
        lib.or_vix_targets.argtypes = [i64, i64, i64, i64, i32, i32, u64, P, P]
        lib.or_findmax.argtypes = [P, i32, i32, P, i64, i64, i64, i32, i32, i32, P]
        lib.or_cell_max.argtypes = [P, i64, i64, i64, i32, i64, i64]
        lib.or_cell_max.restype = i64
        lib.or_layout.argtypes = [P, i64, i64, i64, P]
        lib.or_layout.restype = i64
        lib.or_viewshed_one.argtypes = [P, i64, i64, i64, P, P]
        lib.or_viewshed.argtypes = [P, i64, i64, i64, P, P, i64, i64, P]
        lib.or_viewshed_r3.argtypes = [P, i64, i64, i64, P, P, i64, i64, P]
        lib.or_disk_cells.argtypes = [P, i64, i64]
        lib.or_disk_cells.restype = i64
        lib.or_viewshed_count.argtypes = [P, i64, i64, i64, P, i64, P, P]
        lib.or_greedy.argtypes = [P, P, P, i64, i64, i64, i32, i64, P, P, P, i32]
        lib.or_greedy.restype = i32
        lib.or_greedy_lazy.argtypes = [P, P, P, i64, i64, i64, i32, i64, P, P, P, P, i32]
        lib.or_greedy_lazy.restype = i32
        lib.or_num_threads.restype = i32
        lib.or_set_threads.argtypes = [i32]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _terrain(z):
    z = np.asarray(z)
    if z.dtype != np.int16 or z.ndim != 2:
        raise ValueError("terrain must be a 2-D int16 array")
    z = np.ascontiguousarray(z)
    return z, z.shape[0], z.shape[1]


def observers(x, y, roi, h_t, h_r) -> np.ndarray:
    """Structured observer array {x (column), y (row), roi, h_t, h_r}."""
    x = np.atleast_1d(np.asarray(x))
    o = np.zeros(x.shape[0], OBSERVER_DTYPE)
    o["x"], o["y"], o["roi"], o["h_t"], o["h_r"] = x, y, roi, h_t, h_r
    return o


def num_threads() -> int:
    return int(_load().or_num_threads())


def set_threads(n: int) -> None:
    """Threads of the oracle's parallel loops (timing only)."""
    _load().or_set_threads(int(n))


def philox4x32_10(counter, key) -> np.ndarray:
    """Philox4x32-10 block function (Salmon et al., SC'11)."""
    c = np.ascontiguousarray(counter, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    _load().or_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def los(z, t, p, h_t, h_r) -> bool:
    """Line-of-sight test between observer t=(x,y) and receiver p=(x,y):
    Definitions (line of sight) and section "Terrain visibility"."""
    z, nr, nc = _terrain(z)
    return bool(_load().or_los(_ptr(z), nr, nc, nc, int(t[0]), int(t[1]),
                               int(p[0]), int(p[1]), int(h_t), int(h_r)))


def vix(z, roi, h_t, h_r, K, seed, rows=None) -> np.ndarray:
    """Estimated visibility index (count of K random receivers visible):
    stage Vix of "The multiple transmitter siting process"."""
    z, nr, nc = _terrain(z)
    r0, r1 = (0, nr) if rows is None else rows
    out = np.zeros((nr, nc), np.uint8)
    _load().or_vix(_ptr(z), nr, nc, nc, int(roi), int(h_t), int(h_r), int(K),
                   C.c_uint64(int(seed)), _ptr(out), int(r0), int(r1))
    return out


def vix_rows(z, roi, h_t, h_r, K, seed, rows) -> np.ndarray:
    """The counts of vix() on the listed rows only: (len(rows), ncols)."""
    z, nr, nc = _terrain(z)
    rows = np.ascontiguousarray(rows, np.int64)
    if len(rows) and (rows.min() < 0 or rows.max() >= nr):
        raise ValueError("row outside the terrain")
    out = np.zeros((len(rows), nc), np.uint8)
    _load().or_vix_rowlist(_ptr(z), nr, nc, nc, int(roi), int(h_t), int(h_r), int(K),
                           C.c_uint64(int(seed)), _ptr(rows), len(rows), _ptr(out))
    return out


def vix_targets(nrows, ncols, x, y, roi, K, seed):
    """The K receivers drawn for post (x, y); -1 marks a failed draw."""
    tx = np.zeros(K, np.int64)
    ty = np.zeros(K, np.int64)
    _load().or_vix_targets(int(nrows), int(ncols), int(x), int(y), int(roi), int(K),
                           C.c_uint64(int(seed)), _ptr(tx), _ptr(ty))
    return tx, ty


def findmax(key, z, grid_r, grid_c, k, stride=1) -> np.ndarray:
    """Per-block top-k candidates: stage Findmax.  uint8 keys rank by
    (key desc, z desc, index asc); float32 keys score the cells of a stride
    grid, rank by (key desc, cell index asc) and return each cell's highest
    post."""
    z, nr, nc = _terrain(z)
    key = np.ascontiguousarray(key)
    if key.dtype == np.uint8:
        kt = 0
        stride = 1
    elif key.dtype == np.float32:
        kt = 1
    else:
        raise ValueError("key must be uint8 or float32")
    out = np.zeros(grid_r * grid_c * k, np.int64)
    _load().or_findmax(_ptr(key), kt, int(stride), _ptr(z), nr, nc, nc, int(grid_r),
                       int(grid_c), int(k), _ptr(out))
    return out


def cell_max(z, stride):
    """Highest post (elevation desc, index asc) of every stride x stride cell,
    as linear indices, cells in row-major order."""
    z, nr, nc = _terrain(z)
    lib = _load()
    R, C_ = -(-nr // stride), -(-nc // stride)
    return np.array([lib.or_cell_max(_ptr(z), nr, nc, nc, int(stride), i, j)
                     for i in range(R) for j in range(C_)], np.int64)


def layout(obs, nrows, ncols) -> np.ndarray:
    """Window-bitmap offsets (in 64-bit words) of each observer."""
    obs = np.ascontiguousarray(obs, OBSERVER_DTYPE)
    off = np.zeros(len(obs) + 1, np.int64)
    _load().or_layout(_ptr(obs), len(obs), int(nrows), int(ncols), _ptr(off))
    return off


def viewshed(z, obs, i0=0, i1=None, out=None):
    """Window bitmaps of observers [i0, i1): stage Viewshed.  Returns
    (bitmaps, offsets) with offsets over all observers; `out` (uint64, the
    total words long) receives the windows in place of a new array."""
    z, nr, nc = _terrain(z)
    obs = np.ascontiguousarray(obs, OBSERVER_DTYPE)
    off = layout(obs, nr, nc)
    i1 = len(obs) if i1 is None else i1
    if out is None:
        bm = np.zeros(int(off[-1]), np.uint64)
    else:
        if out.dtype != np.uint64 or out.size < off[-1] or not out.flags.c_contiguous:
            raise ValueError("out must be a contiguous uint64 array of the total words")
        bm = out
    _load().or_viewshed(_ptr(z), nr, nc, nc, _ptr(obs), _ptr(off), int(i0), int(i1), _ptr(bm))
    return bm, off


def viewshed_r3(z, obs, i0=0, i1=None):
    """Exact per-cell viewsheds (every disk cell by its own line of sight,
    the R3 family) of observers [i0, i1), in the layout of viewshed()."""
    z, nr, nc = _terrain(z)
    obs = np.ascontiguousarray(obs, OBSERVER_DTYPE)
    off = layout(obs, nr, nc)
    i1 = len(obs) if i1 is None else i1
    bm = np.zeros(int(off[-1]), np.uint64)
    _load().or_viewshed_r3(_ptr(z), nr, nc, nc, _ptr(obs), _ptr(off), int(i0), int(i1), _ptr(bm))
    return bm, off


def viewshed_one(z, ob) -> np.ndarray:
    """Window bitmap of one observer, shaped (rows, words)."""
    z, nr, nc = _terrain(z)
    ob = np.ascontiguousarray(np.atleast_1d(ob), OBSERVER_DTYPE)
    o = ob[0]
    R = int(o["roi"])
    ylo, yhi = max(0, int(o["y"]) - R), min(nr - 1, int(o["y"]) + R)
    xlo, xhi = max(0, int(o["x"]) - R), min(nc - 1, int(o["x"]) + R)
    nw = (xhi >> 6) - (xlo >> 6) + 1
    bm = np.zeros((yhi - ylo + 1, nw), np.uint64)
    _load().or_viewshed_one(_ptr(z), nr, nc, nc, _ptr(ob), _ptr(bm))
    return bm


def viewshed_count(z, obs):
    """(visible cells, in-disk in-terrain cells) per observer: the numerator
    and denominator of the visibility index (Definitions)."""
    z, nr, nc = _terrain(z)
    obs = np.ascontiguousarray(obs, OBSERVER_DTYPE)
    vis = np.zeros(len(obs), np.uint32)
    cells = np.zeros(len(obs), np.uint32)
    _load().or_viewshed_count(_ptr(z), nr, nc, nc, _ptr(obs), len(obs), _ptr(vis), _ptr(cells))
    return vis, cells


def visibility_index(z, obs) -> np.ndarray:
    """Exact visibility index of each observer (Definitions: the fraction of
    the receivers within the ROI that are visible; the observer's own cell is
    not a receiver): (visible - 1) / (cells - 1) from viewshed_count, as the
    float32 quotient of the counts converted to float32 (0 for cells <= 1)."""
    vis, cells = viewshed_count(z, obs)
    num = (vis.astype(np.int64) - 1).astype(np.float32)
    den = (cells.astype(np.int64) - 1).astype(np.float32)
    ok = (vis >= 1) & (cells >= 2)
    out = np.zeros(len(vis), np.float32)
    out[ok] = num[ok] / den[ok]
    return out


def disk_cells(ob, nrows, ncols) -> int:
    ob = np.ascontiguousarray(np.atleast_1d(ob), OBSERVER_DTYPE)
    return int(_load().or_disk_cells(_ptr(ob), int(nrows), int(ncols)))


def greedy(bitmaps, offsets, obs, nrows, ncols, max_obs, target_cells, lazy=False,
           intervisible=False):
    """Greedy siting: stage Site (lazy=True uses the stage's optimisation
    that gains never grow).  intervisible=True: after the first pick only
    candidates whose post lies in the cumulative viewshed compete.  Returns
    (selected, gains, cumulative[, evals])."""
    obs = np.ascontiguousarray(obs, OBSERVER_DTYPE)
    bitmaps = np.ascontiguousarray(bitmaps, np.uint64)
    offsets = np.ascontiguousarray(offsets, np.int64)
    W = (ncols + 63) // 64
    cum = np.zeros((nrows, W), np.uint64)
    sel = np.zeros(max(max_obs, 1), np.int64)
    gains = np.zeros(max(max_obs, 1), np.int64)
    lib = _load()
    if lazy:
        ev = np.zeros(1, np.int64)
        t = lib.or_greedy_lazy(_ptr(bitmaps), _ptr(offsets), _ptr(obs), len(obs), int(nrows),
                               int(ncols), int(max_obs), int(target_cells), _ptr(cum),
                               _ptr(sel), _ptr(gains), _ptr(ev), int(bool(intervisible)))
        return sel[:t].copy(), gains[:t].copy(), cum, int(ev[0])
    t = lib.or_greedy(_ptr(bitmaps), _ptr(offsets), _ptr(obs), len(obs), int(nrows), int(ncols),
                      int(max_obs), int(target_cells), _ptr(cum), _ptr(sel), _ptr(gains),
                      int(bool(intervisible)))
    return sel[:t].copy(), gains[:t].copy(), cum


def block_grid(n: int, roi: int) -> int:
    """The paper's block count per side, G = round(N / floor(ROI/3)) (stage
    Findmax: blocks of width ROI/3; reproduces Tables 1-3)."""
    w = roi // 3
    return int((2 * n + w) // (2 * w))
