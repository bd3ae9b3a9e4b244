"""Sensitivity of siting to lowered data accuracy (the paper's future work).

Site on a degraded terrain and score the chosen observers on the full one:
  - quantised elevations: z_q = q * floor(z / q) for a step of q metres;
  - coarsened grid: every f-th post in both directions, the ROI divided by f
    (FINDMAX keeps the same block grid and k), the chosen posts mapped back
    to full-resolution positions (x*f, y*f).
The score is the area of the union of the chosen observers' viewsheds on the
full terrain (their exact sweep viewsheds there, united by SITE over just
those observers, whose gains then sum to the union).

    python -m paper_2006_16783_amd.accuracy --config plain_1000
    python -m paper_2006_16783_amd.accuracy --config batched_4096 --quant 1,10,50 --coarsen 2,4

Host logic only: every stage runs in the library's kernels; the degraded
terrains are prepared with tensor arithmetic on the device.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import sys
import time

import numpy as np

from . import _lib as L
from . import pipeline as P


def union_area(z, xs, ys, cfg) -> int:
    """Cells of the full terrain z seen by observers at (xs, ys) with the
    configuration's ROI and heights."""
    import torch
    nr, nc = z.shape
    obs = np.zeros(len(xs), L.OBSERVER_DTYPE)
    obs["x"], obs["y"] = xs, ys
    obs["roi"], obs["h_t"], obs["h_r"] = cfg.roi, cfg.h_t, cfg.h_r
    if len(obs) == 0:
        return 0
    off = L.siting_viewshed_layout(obs, nr, nc)
    obs_d = L.observers_to_device(obs, z.device)
    off_d = torch.from_numpy(off).to(z.device)
    bm = L.siting_viewshed_batch(z, obs_d, off_d, cfg.roi)
    _, gains, nsel, _ = L.siting_greedy(bm, off_d, obs_d, nr, nc, len(obs), nr * nc)
    return int(gains[:int(nsel.item())].sum().item())


def site_degraded(z, cfg, quant=1, coarsen=1):
    """Sites on the degraded terrain; returns the chosen full-resolution
    positions and the pass time in seconds."""
    import torch
    zd = z
    if quant > 1:
        zd = (torch.div(zd, quant, rounding_mode="floor") * quant).to(torch.int16)
    c = cfg
    if coarsen > 1:
        zd = zd[::coarsen, ::coarsen].contiguous()
        nc_ = int(zd.shape[0])
        c = dataclasses.replace(cfg, n=nc_, roi=max(1, cfg.roi // coarsen),
                                grid=min(cfg.grid, nc_))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = P.run(zd, c, timing=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    sel = res.observers[res.selected]
    xs = sel["x"].astype(np.int64) * coarsen
    ys = sel["y"].astype(np.int64) * coarsen
    return xs, ys, dt, res


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", default="plain_1000")
    ap.add_argument("--quant", default="1,2,5,10,20,50", help="elevation steps in metres")
    ap.add_argument("--coarsen", default="2,4", help="grid subsampling factors")
    args = ap.parse_args(argv)
    import torch
    from synth import fbm_torch
    cfg = P.CONFIGS[args.config]
    z = fbm_torch(cfg.n, cfg.beta, cfg.zmax, cfg.seed, device="cuda")
    nr, nc = z.shape
    rows = []
    variants = [(int(q), 1) for q in args.quant.split(",") if q] + \
               [(1, int(f)) for f in args.coarsen.split(",") if f]
    if (1, 1) not in variants:
        variants.insert(0, (1, 1))
    base = None
    for q, f in variants:
        xs, ys, dt, res = site_degraded(z, cfg, q, f)
        area = union_area(z, xs, ys, cfg)
        if (q, f) == (1, 1):
            base = area
            # scoring the exact run's own choice reproduces its coverage
            assert area == res.coverage_cells, (area, res.coverage_cells)
        rows.append({"quant_m": q, "coarsen": f, "observers": int(len(xs)),
                     "coverage_frac": area / (nr * nc), "siting_s": dt})
    for r in rows:
        r["coverage_diff_pp"] = 100.0 * (r["coverage_frac"] - base / (nr * nc))
    out = {"config": cfg.name, "n": cfg.n, "roi": cfg.roi, "max_obs": cfg.max_obs,
           "variants": rows}
    print(json.dumps(out), flush=True)
    return out


if __name__ == "__main__":
    sys.exit(0 if main() else 1)
