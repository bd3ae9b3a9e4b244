"""Siting pipeline driver: VIX -> FINDMAX -> VIEWSHED -> SITE on one GPU
(section "The multiple transmitter siting process").

Host logic only: it chains the C-ABI calls of libsiting on torch's current
stream, moves the small candidate list to the host to build observer
records and the bitmap layout, and times every stage with events on that
stream (the paper's table rows: estimated visibility indexes, potential
transmitters, viewsheds, top transmitters).
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field, asdict

import numpy as np

from . import _lib as L


@dataclass
class SitingConfig:
    name: str
    n: int                 # terrain side (square terrains)
    beta: float            # fBm spectral exponent
    zmax: int              # elevation range 0..zmax
    seed: int              # terrain seed
    roi: int
    h_t: int
    h_r: int
    K: int                 # VIX receivers per post
    grid: int              # FINDMAX blocks per side
    k: int                 # candidates kept per block
    max_obs: int           # SITE observer cap
    target_frac: float     # SITE coverage target (fraction of all posts)
    vix_seed: int = 12345
    intervisible: bool = False  # SITE: every pick after the first seen by an earlier one
    site_batch: int | None = None  # SITE rounds over the GPU with this batch (None: by ROI)

    def to_dict(self):
        return asdict(self)


# The workloads the build is measured and tested on (square fBm terrains).
CONFIGS = {
    # 1000^2, ROI 100, 10x10 blocks of 10 candidates, SITE to 100 observers
    "plain_1000": SitingConfig("plain_1000", 1000, 2.4, 1000, 1, 100, 10, 10, 10, 10, 10, 100, 1.0),
    # 4096^2, ROI 200, 50 receivers, 50x50 blocks x 4 = 10000 tentative
    # observers, SITE to 2000 observers or 90% coverage
    "batched_4096": SitingConfig("batched_4096", 4096, 2.4, 2000, 1, 200, 10, 10, 50, 50, 4,
                                 2000, 0.90),
    # 46400^2 (2.15e9 posts), ROI 100, 64x64 blocks x 20, SITE to 4096
    "full_46400": SitingConfig("full_46400", 46400, 2.4, 4000, 1, 100, 10, 10, 10, 64, 20,
                               4096, 1.0),
    # the paper's billion-post runs (Tables 2 and 3) as synthetic stand-ins:
    # its terrain sizes and elevation spans, h_t = 100, h_r = 10, blocks of
    # side floor(R/3) with 20 candidates each, SITE to the paper's observer
    # counts
    "east_32000_r500": SitingConfig("east_32000_r500", 32000, 2.4, 507, 1, 500, 100, 10, 10,
                                    193, 20, 6543, 1.0),
    "east_32000_r1000": SitingConfig("east_32000_r1000", 32000, 2.4, 507, 1, 1000, 100, 10, 10,
                                     96, 20, 5000, 1.0),
    "west_46400_r1000": SitingConfig("west_46400_r1000", 46400, 2.4, 2706, 1, 1000, 100, 10, 10,
                                     139, 20, 5647, 1.0),
    "west_46400_r2000": SitingConfig("west_46400_r2000", 46400, 2.4, 2706, 1, 2000, 100, 10, 10,
                                     70, 20, 3347, 1.0),
}


@dataclass
class SitingResult:
    selected: np.ndarray
    gains: np.ndarray
    candidates: np.ndarray
    observers: np.ndarray
    offsets: np.ndarray
    coverage_cells: int
    stage_ms: dict = field(default_factory=dict)
    cell_tests: int = 0
    schedule: tuple | None = None
    # with run(..., keep=True): the device tensors of the pass (FINDMAX key,
    # window bitmaps, cumulative viewshed), for checking its outputs
    key: object = None
    bitmaps: object = None
    cumulative: object = None


def site_batch(cfg: SitingConfig) -> int:
    """SITE's parallel-round batch for the workload, 0 for one-workgroup rounds.
    Windows above one wavefront batch (ROI from 128) are evaluated faster by
    many workgroups per round (measured: ROI 200 147 -> 66 ms, ROI 1000
    24.8 -> 0.63 s); at ROI 100 one workgroup is faster (17.6 against 75 ms).
    Intervisibility runs in the one-workgroup kernel."""
    if cfg.site_batch is not None:
        return cfg.site_batch
    if cfg.intervisible or cfg.roi < 128:
        return 0
    return 512 if cfg.roi >= 500 else 256


def target_cells(frac: float, nrows: int, ncols: int) -> int:
    if frac >= 1.0:
        return nrows * ncols
    return int(math.ceil(frac * nrows * ncols))


def disk_cell_counts(obs: np.ndarray, nrows: int, ncols: int) -> np.ndarray:
    """In-terrain ROI-disk cells per observer (the cell-tests of a viewshed),
    counted row by row on the host for the throughput metric."""
    out = np.zeros(len(obs), np.int64)
    for R in np.unique(obs["roi"]):
        R = int(R)
        sel_all = np.nonzero(obs["roi"] == R)[0]
        dy = np.arange(-R, R + 1)
        half = np.floor(np.sqrt(np.maximum(R * R - dy * dy, 0))).astype(np.int64)
        # exact integer square root correction
        half -= (half * half > R * R - dy * dy)
        half += ((half + 1) * (half + 1) <= R * R - dy * dy)
        # observers in chunks of about 2^23 row entries
        step = max(1, (1 << 23) // (2 * R + 1))
        for c0 in range(0, len(sel_all), step):
            sel = sel_all[c0:c0 + step]
            x = obs["x"][sel].astype(np.int64)[:, None]
            y = obs["y"][sel].astype(np.int64)[:, None]
            rows = y + dy[None, :]
            lo = np.maximum(x - half[None, :], 0)
            hi = np.minimum(x + half[None, :], ncols - 1)
            cnt = np.where((rows >= 0) & (rows < nrows), np.maximum(hi - lo + 1, 0), 0)
            out[sel] = cnt.sum(axis=1)
    return out


_QUAD_STEPS: dict = {}


def _quadrant_ray_steps(eu: int, ev: int, R: int) -> int:
    """Ray steps that test a cell in one quadrant of a window (rays to the
    far sides u = eu and v = ev; each ray stops when its nearest cell leaves
    the ROI disk).  Geometry only, independent of the terrain.  Along a ray
    of n major steps and minor extent mn, step k lands at minor offset
    m(k) = floor((2*k*mn + n) / (2n)), so k^2 + m(k)^2 grows with k and the
    ray's steps are the k <= n with k^2 + m(k)^2 <= R^2: the largest such k,
    found from a float estimate corrected by exact integer tests."""
    key = (eu, ev, R)
    if key in _QUAD_STEPS:
        return _QUAD_STEPS[key]
    if eu < 1:
        _QUAD_STEPS[key] = 0
        return 0
    rho = np.arange(eu + ev, dtype=np.int64)
    du = np.where(rho <= ev, eu, eu - (rho - ev))
    dv = np.where(rho <= ev, rho, ev)
    n = np.maximum(du, dv)
    mn = np.minimum(du, dv)

    def ok(k):
        m = (2 * k * mn + n) // (2 * n)
        return (k >= 1) & (k <= n) & (k * k + m * m <= R * R)

    k = np.minimum(n, np.floor(R / np.sqrt(1.0 + (mn / n) ** 2)).astype(np.int64))
    for _ in range(4):
        k = np.where(ok(k + 1), k + 1, k)
    for _ in range(4):
        k = np.where((k >= 1) & ~ok(k), k - 1, k)
    assert ok(k).sum() == (k >= 1).sum() and not ok(k + 1).any()
    tot = int(k.sum())
    _QUAD_STEPS[key] = tot
    return tot


def ray_step_counts(obs: np.ndarray, nrows: int, ncols: int) -> np.ndarray:
    """Algorithmic ray steps of each observer's viewshed sweep (the unit of
    the viewshed kernel's roofline)."""
    out = np.zeros(len(obs), np.int64)
    for i, o in enumerate(obs):
        x, y, R = int(o["x"]), int(o["y"]), int(o["roi"])
        ex_p, ex_m = min(ncols - 1, x + R) - x, x - max(0, x - R)
        ey_p, ey_m = min(nrows - 1, y + R) - y, y - max(0, y - R)
        out[i] = (_quadrant_ray_steps(ex_p, ey_p, R) + _quadrant_ray_steps(ey_p, ex_m, R) +
                  _quadrant_ray_steps(ex_m, ey_m, R) + _quadrant_ray_steps(ey_m, ex_p, R))
    return out


class _Timer:
    def __init__(self, enabled=True):
        import torch
        self.torch = torch
        self.enabled = enabled
        self.events = []

    def mark(self, name):
        if not self.enabled:
            return
        e = self.torch.cuda.Event(enable_timing=True)
        e.record()
        self.events.append((name, e))

    def result(self):
        if not self.enabled or len(self.events) < 2:
            return {}
        self.events[-1][1].synchronize()
        out = {}
        for (n0, e0), (_, e1) in zip(self.events[:-1], self.events[1:]):
            out[n0] = e0.elapsed_time(e1)
        return out


def run(z, cfg: SitingConfig, key=None, key_stride=1, sched=None, timing=True,
        surrogate=None, keep=False, progress=None) -> SitingResult:
    """One pass of the whole siting path over the device terrain z (int16,
    resident in HBM).  The FINDMAX ranking is the VIX count, or `key` (a
    float32 device tensor) when given, or the CNN score of the cells of a
    stride grid when surrogate=(params, stride) is given (computed inside the
    timed pass).  keep=True also returns the pass's device tensors (no extra
    work is enqueued).  progress(text): called when each stage has finished
    (the host waits for it), for passes that run for minutes."""
    import torch
    nrows, ncols = z.shape
    dev = z.device
    T = _Timer(timing)
    if progress is not None:
        t_start = time.perf_counter()
        mark0 = T.mark

        def mark(name):
            torch.cuda.synchronize()
            if T.events:
                progress(f"{T.events[-1][0]} done at {time.perf_counter() - t_start:.1f} s")
            mark0(name)
        T.mark = mark
    T.mark("vix" if key is None and surrogate is None else "score")
    if surrogate is not None:
        params, key_stride = surrogate
        key = L.siting_cnn_score_terrain(params, z, key_stride)
    elif key is None:
        key = L.siting_vix(z, cfg.roi, cfg.h_t, cfg.h_r, cfg.K, cfg.vix_seed)
    T.mark("findmax")
    cand = L.siting_findmax(key, z, cfg.grid, cfg.grid, cfg.k, key_stride=key_stride)
    T.mark("layout")
    cand_h = cand.cpu().numpy()
    cand_h = cand_h[cand_h >= 0]
    obs = np.zeros(len(cand_h), L.OBSERVER_DTYPE)
    obs["x"] = cand_h % ncols
    obs["y"] = cand_h // ncols
    obs["roi"], obs["h_t"], obs["h_r"] = cfg.roi, cfg.h_t, cfg.h_r
    off = L.siting_viewshed_layout(obs, nrows, ncols)
    obs_d = L.observers_to_device(obs, dev)
    off_d = torch.from_numpy(off).to(dev)
    T.mark("viewshed")
    bm = L.siting_viewshed_batch(z, obs_d, off_d, cfg.roi, sched=sched)
    T.mark("site")
    sel, gains, nsel, cum = L.siting_greedy(bm, off_d, obs_d, nrows, ncols, cfg.max_obs,
                                            target_cells(cfg.target_frac, nrows, ncols),
                                            intervisible=cfg.intervisible,
                                            parallel=site_batch(cfg))
    T.mark("d2h")
    m = int(nsel.item())
    sel_h = sel[:m].cpu().numpy()
    gains_h = gains[:m].cpu().numpy()
    T.mark("end")
    res = SitingResult(selected=sel_h, gains=gains_h, candidates=cand_h, observers=obs,
                       offsets=off, coverage_cells=int(gains_h.sum()), stage_ms=T.result(),
                       schedule=None if sched is None else sched.as_tuple())
    if keep:
        res.key, res.bitmaps, res.cumulative = key, bm, cum
    return res
