"""How far the ray sweep's viewsheds are from exact line of sight.

The sweep (stage Viewshed) marks, along each ray to the window boundary, the
cell nearest the ray and tests it against the ray's horizon; exact per-cell
line of sight (the R3 family the paper cites as prior art) tests every disk
cell by its own segment.  The paper uses the sweep and does not quantify the
difference.  This tool runs both kernels on the same candidates and reports
the cells each marks visible that the other does not.

    python -m paper_2006_16783_amd.r3_compare --config plain_1000
    python -m paper_2006_16783_amd.r3_compare --config full_46400 --sample 2048

Host logic only: candidates come from the siting path's VIX and FINDMAX on
the configuration's synthetic terrain; both viewsheds run on the device.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import _lib as L
from . import pipeline as P


def compare(z, obs, rmax):
    """Per-observer counts (sweep only, exact only, both, disk cells) and the
    two kernels' times in ms."""
    import torch
    nr, nc = z.shape
    off = L.siting_viewshed_layout(obs, nr, nc)
    obs_d = L.observers_to_device(obs, z.device)
    off_d = torch.from_numpy(off).to(z.device)
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    e[0].record()
    r2 = L.siting_viewshed_batch(z, obs_d, off_d, rmax)
    e[1].record()
    r3 = L.siting_viewshed_r3(z, obs_d, off_d)
    e[2].record()
    torch.cuda.synchronize()
    a = r2.cpu().numpy().view(np.uint64)[:off[-1]]
    b = r3.cpu().numpy().view(np.uint64)[:off[-1]]
    def per_observer(words):
        # sums over each observer's words (an empty window sums to 0)
        cs = np.concatenate([[0], np.cumsum(words.astype(np.int64))])
        return cs[off[1:]] - cs[off[:-1]]

    out = {
        "sweep_only": per_observer(np.bitwise_count(a & ~b)),
        "exact_only": per_observer(np.bitwise_count(b & ~a)),
        "both": per_observer(np.bitwise_count(a & b)),
        "disk_cells": P.disk_cell_counts(obs, nr, nc),
    }
    return out, e[0].elapsed_time(e[1]), e[1].elapsed_time(e[2])


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", default="plain_1000")
    ap.add_argument("--sample", type=int, default=0,
                    help="compare this many candidates, evenly spaced (0: all)")
    args = ap.parse_args(argv)
    import torch
    from synth import fbm_torch
    cfg = P.CONFIGS[args.config]
    z = fbm_torch(cfg.n, cfg.beta, cfg.zmax, cfg.seed, device="cuda")
    # the configuration's candidates (VIX, then FINDMAX)
    cnt = L.siting_vix(z, cfg.roi, cfg.h_t, cfg.h_r, cfg.K, cfg.vix_seed)
    cand = L.siting_findmax(cnt, z, cfg.grid, cfg.grid, cfg.k).cpu().numpy()
    del cnt
    cand = cand[cand >= 0]
    obs = np.zeros(len(cand), L.OBSERVER_DTYPE)
    obs["x"], obs["y"] = cand % cfg.n, cand // cfg.n
    obs["roi"], obs["h_t"], obs["h_r"] = cfg.roi, cfg.h_t, cfg.h_r
    if args.sample and args.sample < len(obs):
        obs = obs[np.linspace(0, len(obs) - 1, args.sample).astype(np.int64)]
    t0 = time.perf_counter()
    c, t2, t3 = compare(z, obs, cfg.roi)
    tot = {k: int(v.sum()) for k, v in c.items()}
    vis3 = tot["both"] + tot["exact_only"]
    vis2 = tot["both"] + tot["sweep_only"]
    per = (c["sweep_only"] + c["exact_only"]) / np.maximum(c["disk_cells"], 1)
    out = {
        "config": cfg.name, "observers": int(len(obs)), "roi": cfg.roi,
        "h_t": cfg.h_t, "h_r": cfg.h_r, "disk_cells": tot["disk_cells"],
        "visible_exact": vis3, "visible_sweep": vis2,
        "sweep_only": tot["sweep_only"], "exact_only": tot["exact_only"],
        "disagree_frac_of_disk": (tot["sweep_only"] + tot["exact_only"]) / tot["disk_cells"],
        "disagree_frac_of_visible": (tot["sweep_only"] + tot["exact_only"]) / max(vis3, 1),
        "per_observer_disagree_frac": {"median": float(np.median(per)),
                                       "p90": float(np.quantile(per, 0.9)),
                                       "max": float(per.max())},
        "sweep_ms": t2, "exact_ms": t3,
        "sweep_cell_tests_per_s": tot["disk_cells"] / (t2 / 1e3),
        "exact_cell_tests_per_s": tot["disk_cells"] / (t3 / 1e3),
        "host_s": time.perf_counter() - t0,
    }
    print(json.dumps(out), flush=True)
    return out


if __name__ == "__main__":
    sys.exit(0 if main() else 1)
