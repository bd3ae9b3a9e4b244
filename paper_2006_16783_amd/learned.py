"""Learned-ranking experiment: train the CNN on exact visibility indexes of
seeded fBm terrains, then compare, on held-out terrains, siting with the
plain sampled-VIX ranking, with the CNN ranking and with a plain elevation
ranking (coverage at a fixed observer count, wall time), and the rank
correlation of the CNN with the exact visibility index.

Default workload: 4096^2 terrains, exponent drawn from [2.0, 2.8] per seed,
0-2000 m, ROI 100, heights 10/10; seeds 0-31 train, 32-39 test; FINDMAX on
the paper's block rule (round(4096 / floor(100/3)) = 124 blocks per side,
20 per block); SITE to 1000 observers.

    python -m paper_2006_16783_amd.learned [--quick] [--save]
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--train-seeds", type=int, default=32)
    ap.add_argument("--test-seeds", type=int, default=8)
    ap.add_argument("--samples", type=int, default=32768)
    ap.add_argument("--epochs", type=int, default=4)
    ap.add_argument("--batch", type=int, default=512)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--stride", type=int, default=8)
    ap.add_argument("--observers", type=int, default=1000)
    ap.add_argument("--quick", action="store_true", help="small smoke configuration")
    ap.add_argument("--save", action="store_true", help="store the trained weights in the package")
    ap.add_argument("--out", default=None, help="also write weights and summary to this folder")
    args = ap.parse_args(argv)
    if args.quick:
        args.n, args.train_seeds, args.test_seeds, args.samples, args.epochs = 1024, 4, 2, 8192, 2

    import torch
    from . import _lib as L
    from . import pipeline as P
    from . import surrogate as SG

    def log(*a):
        print(*a, file=sys.stderr, flush=True)

    roi, h = 100, 10
    t0 = time.perf_counter()
    train_ds = SG.make_dataset(range(args.train_seeds), args.n, args.samples, roi, h)
    test_ds = SG.make_dataset(range(args.train_seeds, args.train_seeds + args.test_seeds), args.n,
                              args.samples, roi, h)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    log(f"[learned] data: {args.train_seeds}+{args.test_seeds} terrains, {t_data:.1f} s")

    res = SG.train(train_ds, epochs=args.epochs, batch=args.batch, lr=args.lr, log=log)
    log(f"[learned] trained {res.steps} steps in {res.seconds:.1f} s; losses {res.losses}")
    untrained = torch.from_numpy(SG.init_params(0)).cuda()

    g = round(args.n / (roi // 3))
    cfg = P.SitingConfig("learned", args.n, 2.4, 2000, 0, roi, h, h, 10, g, 20, args.observers, 1.0)
    per = []
    for i, z in enumerate(test_ds.terrains):
        pred = SG.predict(res.params, z, test_ds.centres[i]).cpu().numpy()
        pred0 = SG.predict(untrained, z, test_ds.centres[i]).cpu().numpy()
        lab = test_ds.labels[i].cpu().numpy()
        cnt = L.siting_vix(z, roi, h, h, 10, 12345)
        vix = cnt.flatten()[test_ds.centres[i]].cpu().numpy().astype(np.float64) / 10.0
        cmp_ = SG.siting_compare(z, cfg, res.params, args.stride)
        row = {"spearman_cnn": SG.spearman(pred, lab), "spearman_untrained": SG.spearman(pred0, lab),
               "spearman_vix": SG.spearman(vix, lab),
               "mse_cnn": float(np.mean((pred - lab) ** 2)), **cmp_}
        per.append(row)
        log(f"[learned] test {i}: rho cnn {row['spearman_cnn']:.3f} vix {row['spearman_vix']:.3f}; "
            f"coverage plain {cmp_['plain']['coverage']:.4f} cnn {cmp_['surrogate']['coverage']:.4f} "
            f"elev {cmp_['elevation']['coverage']:.4f}")

    def mean(key, sub=None):
        return float(np.mean([r[key] if sub is None else r[key][sub] for r in per]))

    summary = {
        "workload": f"{args.n}^2 fBm beta U[2.0,2.8], 0-2000 m, ROI {roi}, h {h}/{h}, "
                    f"FINDMAX {g}x{g} x 20, SITE to {args.observers}, CNN score stride {args.stride}",
        "train": {"terrains": args.train_seeds, "samples_per_terrain": args.samples,
                  "epochs": args.epochs, "steps": res.steps, "seconds": res.seconds,
                  "losses": res.losses, "data_seconds": t_data},
        "test_terrains": args.test_seeds,
        "spearman_cnn": mean("spearman_cnn"), "spearman_untrained": mean("spearman_untrained"),
        "spearman_vix": mean("spearman_vix"), "mse_cnn": mean("mse_cnn"),
        "coverage_plain": mean("plain", "coverage"), "coverage_cnn": mean("surrogate", "coverage"),
        "coverage_elevation": mean("elevation", "coverage"),
        "coverage_diff_pp": 100 * (mean("surrogate", "coverage") - mean("plain", "coverage")),
        "seconds_plain": mean("plain", "seconds"), "seconds_cnn": mean("surrogate", "seconds"),
        "per_terrain": per,
    }
    meta = {k: v for k, v in summary.items() if k != "per_terrain"}
    if args.save:
        SG.save_weights(res.params, meta)
    if args.out:
        import os
        SG.save_weights(res.params, meta, path=os.path.join(args.out, "surrogate_r100_h10.npy"))
    print(json.dumps(summary), flush=True)
    return summary


if __name__ == "__main__":
    main()
