"""Learned ranking: train the CNN of libsiting on exact visibility indexes
and use its score as the FINDMAX key.

The visibility index of a post (Definitions: the fraction of the receivers
within the ROI that are visible) is computed exactly from the viewshed count
sink: (visible - 1) / (disk cells - 1), the observer's own cell excluded.
Training, inference and the optimiser all run in libsiting's kernels; this
module only samples posts, batches them and keeps score.
"""
from __future__ import annotations

import json
import math
import os
import time
from dataclasses import dataclass, field

import numpy as np

from . import _lib as L
from . import pipeline as P

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "weights", "surrogate_r100_h10.npy")
WEIGHTS_META = os.path.join(HERE, "weights", "surrogate_r100_h10.json")


def init_params(seed: int = 0) -> np.ndarray:
    """He initialisation of the flat parameter vector (fp32)."""
    rng = np.random.default_rng(seed)
    shapes = [("w1", (16, 4, 4)), ("b1", (16,)), ("w2", (16, 3, 3, 16)), ("b2", (16,)),
              ("w3", (32, 3, 3, 16)), ("b3", (32,)), ("wfc", (32,)), ("bfc", (1,))]
    parts = []
    for name, shp in shapes:
        if name.startswith("b"):
            parts.append(np.zeros(int(np.prod(shp))))
        else:
            fan_in = int(np.prod(shp[1:])) if len(shp) > 1 else shp[0]
            parts.append(rng.standard_normal(int(np.prod(shp))) * math.sqrt(2.0 / fan_in))
    theta = np.concatenate(parts).astype(np.float32)
    assert theta.size == L.siting_cnn_param_count()
    return theta


def exact_vi(z, centres, roi: int, h: int):
    """Exact visibility index of the posts `centres` (device int64) on the
    device terrain z, as a device float32 tensor."""
    import torch
    nr, nc = z.shape
    c = centres.cpu().numpy()
    obs = np.zeros(len(c), L.OBSERVER_DTYPE)
    obs["x"], obs["y"] = c % nc, c // nc
    obs["roi"], obs["h_t"], obs["h_r"] = roi, h, h
    vis, cells = L.siting_viewshed_batch(z, L.observers_to_device(obs, z.device), None, roi,
                                         sink=L.SITING_SINK_COUNT)
    return L.siting_visibility_index(vis[:len(c)], cells[:len(c)])


@dataclass
class Dataset:
    terrains: list
    centres: list
    labels: list


def make_dataset(seeds, n_side: int, samples: int, roi: int, h: int, zmax: int = 2000,
                 beta_range=(2.0, 2.8), device="cuda") -> Dataset:
    """Seeded fBm terrains (beta drawn per seed) with `samples` uniformly drawn
    posts each, labelled with their exact visibility index."""
    import torch
    from synth import fbm_torch
    ds = Dataset([], [], [])
    for s in seeds:
        beta = float(np.random.default_rng(1000 + s).uniform(*beta_range))
        z = fbm_torch(n_side, beta, zmax, s, device=device)
        rng = np.random.default_rng(2000 + s)
        c = torch.from_numpy(rng.integers(0, n_side * n_side, size=samples).astype(np.int64)).to(device)
        ds.terrains.append(z)
        ds.centres.append(c)
        ds.labels.append(exact_vi(z, c, roi, h))
    return ds


@dataclass
class TrainResult:
    params: object
    losses: list = field(default_factory=list)
    seconds: float = 0.0
    steps: int = 0


def train(ds: Dataset, epochs: int = 4, batch: int = 512, lr: float = 1e-3, seed: int = 0,
          params=None, log=None) -> TrainResult:
    """Adam on the mean squared error; each step takes one batch from one
    terrain (terrains visited in a seeded random order)."""
    import torch
    dev = ds.terrains[0].device
    theta = torch.from_numpy(init_params(seed) if params is None else params).to(dev)
    m = torch.zeros_like(theta)
    v = torch.zeros_like(theta)
    ws = L.cnn_workspace(batch, dev)
    rng = np.random.default_rng(seed)
    res = TrainResult(params=theta)
    t0 = time.perf_counter()
    step = 0
    for ep in range(epochs):
        order = []
        for ti, c in enumerate(ds.centres):
            perm = rng.permutation(c.numel())
            order += [(ti, perm[i:i + batch]) for i in range(0, len(perm) - batch + 1, batch)]
        rng.shuffle(order)
        ep_loss = []
        for ti, idx in order:
            it = torch.from_numpy(idx).to(dev)
            cen = ds.centres[ti][it].contiguous()
            lab = ds.labels[ti][it].contiguous()
            L.siting_cnn_forward(theta, ds.terrains[ti], cen, ws)
            g, loss = L.siting_cnn_backward(theta, lab, ws)
            step += 1
            L.siting_cnn_adam(theta, m, v, g, step, lr)
            ep_loss.append(loss)
        el = float(torch.stack(ep_loss).mean().cpu())
        res.losses.append(el)
        if log:
            log(f"epoch {ep}: loss {el:.5f} ({step} steps)")
    torch.cuda.synchronize()
    res.seconds = time.perf_counter() - t0
    res.steps = step
    return res


def predict(params, z, centres, batch: int = 4096):
    import torch
    out = []
    ws = L.cnn_workspace(min(batch, centres.numel()), z.device)
    for i in range(0, centres.numel(), batch):
        c = centres[i:i + batch].contiguous()
        if c.numel() != batch and ws.numel() < L.siting_cnn_workspace_size(c.numel()):
            ws = L.cnn_workspace(c.numel(), z.device)
        out.append(L.siting_cnn_forward(params, z, c, ws))
    return torch.cat(out)


def spearman(a: np.ndarray, b: np.ndarray) -> float:
    from scipy.stats import spearmanr
    return float(spearmanr(a, b).statistic)


def siting_compare(z, cfg: P.SitingConfig, params, stride: int, timing=True):
    """Plain (sampled-VIX ranking) against surrogate ranking (CNN score on the
    stride lattice) and an elevation ranking, all with the same exact VIEWSHED
    and SITE.  Returns coverage (fraction of posts) at the configured number
    of observers and the wall time of each run."""
    import torch
    out = {}
    nr, nc = z.shape
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain = P.run(z, cfg, timing=timing)
    torch.cuda.synchronize()
    out["plain"] = {"coverage": plain.coverage_cells / (nr * nc), "seconds": time.perf_counter() - t0,
                    "selected": int(len(plain.selected)), "stage_ms": plain.stage_ms}
    t0 = time.perf_counter()
    score = L.siting_cnn_score_terrain(params, z, stride)
    sur = P.run(z, cfg, key=score, key_stride=stride, timing=timing)
    torch.cuda.synchronize()
    out["surrogate"] = {"coverage": sur.coverage_cells / (nr * nc),
                        "seconds": time.perf_counter() - t0, "selected": int(len(sur.selected)),
                        "stage_ms": sur.stage_ms}
    elev = z.to(torch.float32).contiguous()
    elev_res = P.run(z, cfg, key=elev, key_stride=1, timing=False)
    out["elevation"] = {"coverage": elev_res.coverage_cells / (nr * nc),
                        "selected": int(len(elev_res.selected))}
    return out


def save_weights(params, meta: dict, path: str = WEIGHTS):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    np.save(path, params.cpu().numpy() if hasattr(params, "cpu") else np.asarray(params))
    with open(os.path.splitext(path)[0] + ".json", "w") as f:
        json.dump(meta, f, indent=1)


def load_weights(path: str = WEIGHTS, device="cuda"):
    import torch
    a = np.load(path, allow_pickle=False).astype(np.float32)
    if a.size != L.siting_cnn_param_count():
        raise ValueError(f"{path}: {a.size} parameters, expected {L.siting_cnn_param_count()}")
    return torch.from_numpy(a).to(device)
