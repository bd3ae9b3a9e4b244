#!/usr/bin/env python3
"""Benchmark of the siting path on one MI355X.

Workload (default): the full-scale configuration -- a 46400 x 46400 int16 fBm
terrain (2.15e9 posts, exponent 2.4, 0-4000 m) resident in HBM, ROI 100,
heights 10/10, VIX with 10 receivers per post, FINDMAX on a 64 x 64 block
grid keeping 20 per block (81,920 candidates), SITE greedy to 4096 observers.

One step = one pass of the whole path: VIX -> FINDMAX -> layout -> VIEWSHED
(one persistent launch) -> SITE -> selected list on the host.

Printed: ONE JSON line.  `value` is the viewshed throughput in cell-tests/s
(in-disk in-terrain cells of all candidate viewsheds / viewshed stage time);
`siting_wall_s` is the whole step's wall time (the second half of the
metric).  `roofline` describes the dominant kernel of the step (VIX);
`cpu_baseline` times the oracle on the host cores on a bounded sample;
`site_intervisible` times SITE with intervisibility (every pick after the
first seen by an earlier one) on the last step's windows; `parity` compares
the last timed step with the oracle (every viewshed, the oracle's SITE on its
own bitmaps with and without intervisibility, VIX rows, every FINDMAX block),
and the script exits with status 1 if they differ.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
# 32-bit integer VALU: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (non-packed)
PEAK_INT_TOPS = 256 * 64 * 2.4e9 / 1e12
# integer ALU operations of one line-of-sight step: advance
# the crossing (add, compare, conditional subtract), two address updates,
# interpolate (subtract, two multiplies, add), advance the segment (add),
# compare
VIX_OPS_PER_LOS_STEP = 11
# one viewshed ray step: the line-of-sight step work plus the nearest-cell
# rounding, disk test, horizon slope products and comparisons, bit address
VIEWSHED_OPS_PER_RAY_STEP = 24
# dense bf16 MFMA peak (TFLOP/s) and the ranking CNN's multiply-adds per
# scored cell: conv1 16x16 positions x 16 channels x 16, conv2 7x7 x 16 x 144,
# conv3 3x3 x 32 x 144, FC 32 (212,000 of them reach the output: conv1's
# last row and column feed no conv2 output)
PEAK_BF16_TFLOPS = 2500.0
CNN_MACS_PER_CELL = 16 * 16 * 16 * 16 + 49 * 16 * 144 + 9 * 32 * 144 + 32
CNN_MACS_TO_OUTPUT = 15 * 15 * 16 * 16 + 49 * 16 * 144 + 9 * 32 * 144 + 32


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_hash(names):
    """Sources and compile flags of a kernel (counter records match on it)."""
    from paper_2006_16783_amd import build as B
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_2006_16783_amd", "csrc", n), "rb") as f:
            h.update(f.read())
        if n.endswith(".hip"):
            h.update(" ".join(B.flags_of(n)).encode())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel: str, src_hash: str):
    """HBM bytes per launch of `kernel` from the committed counter summary,
    or None when absent or taken on different kernel sources."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
        e = d.get(kernel)
        if not e or e.get("source_hash") != src_hash:
            return None
        return float(e["bytes_per_launch"])
    except Exception:
        return None


def cpu_baseline_and_parity(z_host, res, cfg, seconds: float, full_seconds: float,
                            inter=None):
    """The oracle on this host's cores, on the outputs of the last timed step
    (`res`, a pass run with keep=True), as both the CPU baseline and the
    parity check of the timed run:
      - viewsheds of the step's candidates in index order (cell-tests/s), each
        window compared with the device's: all of them when they fit in
        `full_seconds`, else a prefix of about `seconds` of work;
      - once every window is computed, the oracle's greedy SITE on its own
        bitmaps against the step's selection and gains (and, given `inter` =
        (selected, gains) of the device's SITE with intervisibility on the
        step's windows, the oracle's intervisible greedy against it);
      - VIX on whole rows (LOS tests/s) against the step's counts;
      - FINDMAX of every block, from the step's counts, against its candidates.
    Returns (cpu_baseline, parity)."""
    import numpy as np
    import oracle
    from paper_2006_16783_amd.pipeline import disk_cell_counts, target_cells
    oracle.build()
    nr, nc = z_host.shape
    obs, off = res.observers, res.offsets
    M = len(obs)
    dev_bm = res.bitmaps.cpu().numpy().view(np.uint64)
    or_bm = np.zeros(int(off[-1]), np.uint64)
    cells_all = disk_cell_counts(obs, nr, nc)
    t_used, done, n, bad_windows = 0.0, 0, 256, 0
    while done < M:
        i1 = min(M, done + n)
        t0 = time.perf_counter()
        oracle.viewshed(z_host, obs, done, i1, out=or_bm)
        dt = time.perf_counter() - t0
        t_used += dt
        a, b = int(off[done]), int(off[i1])
        if not (or_bm[a:b] == dev_bm[a:b]).all():
            for i in range(done, i1):
                bad_windows += int(not (or_bm[off[i]:off[i + 1]] == dev_bm[off[i]:off[i + 1]]).all())
        done = i1
        rate = int(cells_all[:done].sum()) / t_used
        if t_used >= seconds and t_used + int(cells_all[done:].sum()) / rate > full_seconds:
            break
        n = int(max(n, min(M - done, n * 4)))
    cells = int(cells_all[:done].sum())
    vs_rate = cells / t_used
    parity = {"viewsheds": f"{done - bad_windows}/{M}" + ("" if done == M else f" (first {done})"),
              "viewshed_mismatches": bad_windows}
    site_ok = None
    if done == M:
        sel, gains, _, _ = oracle.greedy(or_bm, off, obs, nr, nc, cfg.max_obs,
                                         target_cells(cfg.target_frac, nr, nc), lazy=True)
        site_ok = bool(len(sel) == len(res.selected) and (sel == res.selected).all() and
                       (gains == res.gains).all())
    parity["site"] = site_ok
    if done == M and inter is not None:
        isel, igain, _, _ = oracle.greedy(or_bm, off, obs, nr, nc, cfg.max_obs,
                                          target_cells(cfg.target_frac, nr, nc), lazy=True,
                                          intervisible=True)
        parity["site_intervisible"] = bool(len(isel) == len(inter[0]) and
                                           (isel == inter[0]).all() and
                                           (igain == inter[1]).all())
    del dev_bm, or_bm
    # VIX: whole rows until ~40% of the budget, compared with the step's counts
    rows = 1
    t_vix, tests, bad_rows = 0.0, 0, 0
    r0 = nr // 2
    r_first = r0
    while t_vix < seconds * 0.4:
        t0 = time.perf_counter()
        want = oracle.vix_rows(z_host, cfg.roi, cfg.h_t, cfg.h_r, cfg.K, cfg.vix_seed,
                               np.arange(r0, r0 + rows))
        t_vix += time.perf_counter() - t0
        got = res.key[r0:r0 + rows].cpu().numpy()
        bad_rows += int((got != want).any(axis=1).sum())
        tests += rows * nc * cfg.K
        r0 += rows
        rows *= 2
        if r0 + rows > nr:
            break
    nrows_v = r0 - r_first
    parity["vix_rows"] = f"{nrows_v - bad_rows}/{nrows_v} (rows {r_first}..{r0 - 1})"
    # FINDMAX: every block, ranked by the step's own counts
    key_h = res.key.cpu().numpy()
    cand = oracle.findmax(key_h, z_host, cfg.grid, cfg.grid, cfg.k)
    del key_h
    nblk = cfg.grid * cfg.grid
    want_c = cand[cand >= 0]
    fm_ok = len(want_c) == len(res.candidates) and bool((want_c == res.candidates).all())
    parity["findmax_blocks"] = (f"{nblk}/{nblk}" if fm_ok else
                                f"mismatch ({len(want_c)} vs {len(res.candidates)} candidates)")
    parity["ok"] = bool(bad_windows == 0 and site_ok is not False and bad_rows == 0 and fm_ok
                        and parity.get("site_intervisible", True))
    cpu = {
        "value": vs_rate, "unit": "cell-tests/s", "cores": oracle.num_threads(), "kind": "oracle",
        "sample": f"oracle viewsheds of {done} of the {M} candidates ({cells} cell-tests, "
                  f"{t_used:.1f} s); oracle VIX on {nrows_v} full rows "
                  f"({tests} LOS tests, {t_vix:.1f} s)",
        "vix_los_tests_per_s": tests / t_vix if t_vix > 0 else None,
    }
    return cpu, parity


def cpu_per_core(seconds: float):
    """The oracle's viewshed on one host thread, on the candidates of the
    1000^2 (ROI 100) and 4096^2 (ROI 200) workloads (the first up to
    `seconds`, the second a bounded prefix): cell-tests/s per core, the unit
    of the paper's CPU figures."""
    import numpy as np
    import torch
    import oracle
    import paper_2006_16783_amd as S
    from paper_2006_16783_amd import pipeline as P
    from synth import fbm_torch
    oracle.build()
    out = {}
    before = oracle.num_threads()
    oracle.set_threads(1)
    try:
        for name in ("plain_1000", "batched_4096"):
            cfg = P.CONFIGS[name]
            z = fbm_torch(cfg.n, cfg.beta, cfg.zmax, cfg.seed, device="cuda")
            cnt = S.siting_vix(z, cfg.roi, cfg.h_t, cfg.h_r, cfg.K, cfg.vix_seed)
            cand = S.siting_findmax(cnt, z, cfg.grid, cfg.grid, cfg.k).cpu().numpy()
            cand = cand[cand >= 0]
            obs = oracle.observers(cand % cfg.n, cand // cfg.n, cfg.roi, cfg.h_t, cfg.h_r)
            z_host = z.cpu().numpy()
            done, cells, t_used, n = 0, 0, 0.0, 32
            while done < len(obs) and t_used < seconds:
                sub = obs[done:done + n]
                t0 = time.perf_counter()
                oracle.viewshed(z_host, sub)
                t_used += time.perf_counter() - t0
                cells += int(P.disk_cell_counts(sub, cfg.n, cfg.n).sum())
                done += len(sub)
                n *= 2
            out[name] = {"cell_tests_per_s": cells / t_used, "candidates": done,
                         "of": int(len(obs)), "seconds": t_used}
    finally:
        oracle.set_threads(before)
    out["threads"] = 1
    return out


def intervisible_leg(S, P, last, cfg, nr, nc, reps, dev, plain_site_ms):
    """SITE with intervisibility on the windows of the pass `last` (run with
    keep=True): median of `reps` timed runs after one warm-up; returns the
    summary and (selected, gains) for the oracle check."""
    import numpy as np
    import torch
    obs_d = S.observers_to_device(last.observers)
    off_d = torch.from_numpy(last.offsets).to(dev)
    tgt = P.target_cells(cfg.target_frac, nr, nc)
    ws_g = torch.empty(S.siting_greedy_workspace_size(len(last.observers)), dtype=torch.uint8,
                       device=dev)
    inter_ms = []
    for i in range(1 + reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        isel, igain, inum, _ = S.siting_greedy(last.bitmaps, off_d, obs_d, nr, nc, cfg.max_obs,
                                               tgt, ws=ws_g, intervisible=True)
        e1.record()
        e1.synchronize()
        if i > 0:
            inter_ms.append(e0.elapsed_time(e1))
    im = int(inum.item())
    res = (isel[:im].cpu().numpy(), igain[:im].cpu().numpy())
    out = {"site_ms": float(np.median(inter_ms)), "selected": im,
           "coverage_frac": int(res[1].sum()) / (nr * nc), "plain_site_ms": plain_site_ms,
           "plain_coverage_frac": last.coverage_cells / (nr * nc)}
    log(f"[bench] SITE with intervisibility: {out}")
    return out, res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="full_46400")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle leg (CPU baseline and parity check of the timed run)")
    ap.add_argument("--parity-seconds", type=float, default=120.0,
                    help="oracle viewsheds of every candidate when they fit in this time "
                         "(then SITE is re-run by the oracle too)")
    ap.add_argument("--autotune", action="store_true",
                    help="pick the viewshed schedule with the autotuner before timing")
    ap.add_argument("--schedule-cache", default=None,
                    help="with --autotune: JSON file of tuned schedules to reuse and extend")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one 1 GiB device copy (counter calibration for rocprof)")
    ap.add_argument("--no-intervisible", action="store_true",
                    help="skip the SITE-with-intervisibility leg")
    ap.add_argument("--surrogate-stride", type=int, default=8,
                    help="cell size of the CNN-ranked leg (0 skips that leg)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the siting path runs on a single device)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2006_16783_amd as S
    from paper_2006_16783_amd import pipeline as P
    from synth import fbm_torch

    cfg = P.CONFIGS[args.config]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    log(f"[bench] generating {cfg.n}x{cfg.n} fBm terrain on the device")
    t0 = time.perf_counter()
    z = fbm_torch(cfg.n, cfg.beta, cfg.zmax, cfg.seed, device=dev)
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    log(f"[bench] terrain ready in {gen_s:.1f} s; z range {int(z.min())}..{int(z.max())}")

    if args.copy_calibration:
        a = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    sched = None
    if args.autotune:
        # tune on the real candidate set of one pass
        res0 = P.run(z, cfg, timing=False)
        obs_d = S.observers_to_device(res0.observers)
        off_d = torch.from_numpy(res0.offsets).to(dev)
        bm = torch.empty(int(res0.offsets[-1]), dtype=torch.int64, device=dev)
        if args.schedule_cache:
            from paper_2006_16783_amd import schedule_cache
            sched, hit = schedule_cache.autotune_cached(z, obs_d, off_d, cfg.roi, bm,
                                                        args.schedule_cache)
            log(f"[bench] schedule {sched} ({'cached' if hit else 'autotuned, stored'})")
        else:
            sched, times = S.siting_autotune(z, obs_d, off_d, cfg.roi, bm)
            log(f"[bench] autotuned schedule {sched}: {['%.2f' % t for t in times]} ms")
        del bm

    # paper-scale passes run for minutes: report each finished stage
    prog = (lambda t: log(f"[bench]   {t}")) if cfg.roi >= 500 else None
    for i in range(args.warmup):
        r = P.run(z, cfg, sched=sched, progress=prog)
        log(f"[bench] warmup {i}: {r.stage_ms}")
    torch.cuda.synchronize()
    stage_tot = {}
    results = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        # the last step keeps its device outputs for the parity check (the
        # same work is enqueued either way)
        r = P.run(z, cfg, sched=sched, keep=(i == args.steps - 1), progress=prog)
        results.append(r)
        for k, v in r.stage_ms.items():
            stage_tot[k] = stage_tot.get(k, 0.0) + v
        log(f"[bench] step {i}: {r.stage_ms}")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps
    stage_ms = {k: v / args.steps for k, v in stage_tot.items()}
    last = results[-1]
    nr, nc = z.shape
    cells = int(P.disk_cell_counts(last.observers, nr, nc).sum())
    value = cells / (stage_ms["viewshed"] / 1e3)

    # dominant kernel: VIX.  Exact executed line-of-sight steps from the
    # counting variant (untimed), ALU ops per step as stated above.
    _, los_steps, los_tests, _ = S.siting_vix_stats(z, cfg.roi, cfg.h_t, cfg.h_r, cfg.K,
                                                 cfg.vix_seed)
    vix_s = stage_ms["vix"] / 1e3
    achieved = los_steps * VIX_OPS_PER_LOS_STEP / vix_s / 1e12
    vix_hash = source_hash(["vix.hip", "common.hpp"])
    roofline = {
        "bound": "alu", "kernel": "vix_kernel", "achieved": achieved, "peak": PEAK_INT_TOPS,
        "unit": "Top/s", "frac": achieved / PEAK_INT_TOPS,
        "traffic": traffic_from_profiles("vix_kernel", vix_hash),
        "units_per_launch": {"los_steps": los_steps, "los_tests": los_tests,
                             "ops_per_los_step": VIX_OPS_PER_LOS_STEP},
        "kernel_ms": stage_ms["vix"],
        "hbm_frac": (nr * nc * 3) / vix_s / 1e9 / PEAK_HBM_GBS,
    }
    ray_steps = int(P.ray_step_counts(last.observers, nr, nc).sum())
    vs_s = stage_ms["viewshed"] / 1e3
    vs_ach = ray_steps * VIEWSHED_OPS_PER_RAY_STEP / vs_s / 1e12
    vs_hash = source_hash(["viewshed.hip", "common.hpp"])
    bm_bytes = int(last.offsets[-1]) * 8
    vs_roof = {
        "bound": "alu", "kernel": "viewshed_kernel", "achieved": vs_ach, "peak": PEAK_INT_TOPS,
        "unit": "Top/s", "frac": vs_ach / PEAK_INT_TOPS,
        "traffic": traffic_from_profiles("viewshed_kernel", vs_hash),
        "units_per_launch": {"ray_steps": ray_steps, "cell_tests": cells,
                             "ops_per_ray_step": VIEWSHED_OPS_PER_RAY_STEP},
        "kernel_ms": stage_ms["viewshed"],
        "hbm_frac": (cells * 2 + bm_bytes) / vs_s / 1e9 / PEAK_HBM_GBS,
    }

    # SITE with intervisibility (every pick after the first seen by an earlier
    # one) on the last step's windows, timed on its own
    inter, inter_res = None, None
    if not args.no_intervisible:
        inter, inter_res = intervisible_leg(S, P, last, cfg, nr, nc, args.steps, dev,
                                            stage_ms["site"])

    # surrogate-ranked leg: the same path with the CNN score of the cells of
    # a stride grid as the FINDMAX key (weights trained on 4096^2 terrains)
    sur = None
    if args.surrogate_stride > 0:
        from paper_2006_16783_amd import surrogate as SG
        params = SG.load_weights(device=dev)
        P.run(z, cfg, surrogate=(params, args.surrogate_stride))
        torch.cuda.synchronize()
        sur_tot, sres = {}, None
        t1 = time.perf_counter()
        for i in range(args.steps):
            sres = P.run(z, cfg, surrogate=(params, args.surrogate_stride))
            for k, v in sres.stage_ms.items():
                sur_tot[k] = sur_tot.get(k, 0.0) + v
            log(f"[bench] surrogate step {i}: {sres.stage_ms}")
        torch.cuda.synchronize()
        sur_ms = (time.perf_counter() - t1) * 1e3 / args.steps
        sur = {"siting_wall_s": sur_ms / 1e3, "ms_per_step": sur_ms, "stride": args.surrogate_stride,
               "stage_ms": {k: v / args.steps for k, v in sur_tot.items()},
               "selected": int(len(sres.selected)), "candidates": int(len(sres.observers)),
               "coverage_frac": sres.coverage_cells / (nr * nc),
               "plain_coverage_frac": last.coverage_cells / (nr * nc),
               "coverage_diff_pp": 100.0 * (sres.coverage_cells - last.coverage_cells) / (nr * nc),
               "speedup_vs_plain": ms_per_step / sur_ms,
               "weights": "paper_2006_16783_amd/weights/surrogate_r100_h10.npy"}
        # the scoring kernel against the bf16 MFMA roof
        st = args.surrogate_stride
        cells = ((nr + st - 1) // st) * ((nc + st - 1) // st)
        score_s = sur["stage_ms"]["score"] / 1e3
        ach = cells * 2 * CNN_MACS_PER_CELL / score_s / 1e12
        sur["cnn_roofline"] = {
            "bound": "mfma", "kernel": "cnn_fwd_kernel", "achieved": ach,
            "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s", "frac": ach / PEAK_BF16_TFLOPS,
            "frac_output_macs": ach * CNN_MACS_TO_OUTPUT / CNN_MACS_PER_CELL / PEAK_BF16_TFLOPS,
            "units_per_launch": {"cells": cells, "macs_per_cell": CNN_MACS_PER_CELL,
                                 "macs_to_output_per_cell": CNN_MACS_TO_OUTPUT},
            "kernel_ms": sur["stage_ms"]["score"]}

    cpu = None
    parity = None
    if not args.no_cpu_baseline:
        log("[bench] timing the oracle on the host and checking the last step against it")
        z_host = z.cpu().numpy()
        cpu, parity = cpu_baseline_and_parity(z_host, last, cfg, args.cpu_seconds,
                                              args.parity_seconds, inter=inter_res)
        del z_host
        log(f"[bench] parity {parity}")
        log("[bench] timing the oracle on one host thread (per-core figure)")
        cpu["per_core"] = cpu_per_core(args.cpu_seconds / 3)

    out = {
        "metric": "viewshed cell-tests/s; siting wall-time at 46400², 4096 observers",
        "value": value,
        "unit": "cell-tests/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "siting_wall_s": ms_per_step / 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"{cfg.name}: {cfg.n}x{cfg.n} int16 fBm terrain (beta {cfg.beta}, "
                               f"0-{cfg.zmax} m), ROI {cfg.roi}, h {cfg.h_t}/{cfg.h_r}, VIX K={cfg.K}, "
                               f"FINDMAX {cfg.grid}x{cfg.grid} x {cfg.k}, SITE to {cfg.max_obs}",
                   "candidates": int(len(last.observers)), "selected": int(len(last.selected)),
                   "coverage_frac": last.coverage_cells / (nr * nc), "cell_tests": cells,
                   "parallelism": "single GPU"},
        "stage_ms": stage_ms,
        "terrain_gen_s": gen_s,
        "schedule": None if sched is None else sched.as_tuple(),
        "roofline": roofline,
        "viewshed_roofline": vs_roof,
        "surrogate": sur,
        "site_intervisible": inter,
        "cpu_baseline": cpu,
        "parity": parity,
    }
    print(json.dumps(out), flush=True)
    if parity is not None and not parity["ok"]:
        log("[bench] the timed run differs from the oracle")
        sys.exit(1)


if __name__ == "__main__":
    main()
