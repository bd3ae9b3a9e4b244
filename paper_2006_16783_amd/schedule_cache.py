"""A JSON cache of autotuned viewshed schedules.

`siting_autotune` times every candidate schedule on the caller's observers and
returns the fastest; every schedule gives the same bits, so the choice only
matters for speed and can be reused for similar batches.  This module keeps
those choices in a JSON file keyed by the device, the largest ROI, the batch
size (rounded to a power of two) and the terrain size, so that repeated runs
skip the tuning launches.  It is host logic only: the library itself does no
file I/O.
"""
from __future__ import annotations

import json
import os
import tempfile

from ._lib import Schedule, siting_abi_version, siting_autotune


def cache_key(device: str, rmax: int, n: int, nrows: int, ncols: int) -> str:
    """Entries are shared by batches of the same device, ROI maximum, terrain
    size and power-of-two batch bucket."""
    bucket = 1 << max(0, int(n) - 1).bit_length()
    return f"{device}|abi{siting_abi_version()}|rmax{int(rmax)}|n{bucket}|{int(nrows)}x{int(ncols)}"


def load(path: str) -> dict:
    try:
        with open(path) as f:
            data = json.load(f)
    except (FileNotFoundError, json.JSONDecodeError):
        return {}
    return data if isinstance(data, dict) else {}


def store(path: str, data: dict) -> None:
    """Atomic replace, so that a reader never sees a half-written file."""
    d = os.path.dirname(os.path.abspath(path))
    os.makedirs(d, exist_ok=True)
    fd, tmp = tempfile.mkstemp(prefix=".schedules.", dir=d)
    try:
        with os.fdopen(fd, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except BaseException:
        os.unlink(tmp)
        raise


def autotune_cached(z, obs_dev, offsets_dev, rmax, bitmaps, path, order_dev=None, tune=None):
    """The cached schedule for this batch's key, or a fresh autotune (stored).

    Returns (Schedule, hit).  `tune` replaces `siting_autotune` (same
    signature and result) for callers that time differently."""
    import torch
    nrows, ncols = int(z.shape[0]), int(z.shape[1])
    device = torch.cuda.get_device_name(z.device) if z.is_cuda else str(z.device)
    key = cache_key(device, rmax, int(obs_dev.shape[0]), nrows, ncols)
    data = load(path)
    hit = data.get(key)
    if hit is not None:
        s = Schedule()
        v = [int(x) for x in hit["schedule"]] + [0]  # (entries without ray_per_wave: 0)
        s.waves, s.groups_per_cu, s.stage_rmax, s.ray_per_wave = v[:4]
        return s, True
    tune = tune or siting_autotune
    best, times = tune(z, obs_dev, offsets_dev, rmax, bitmaps, order_dev=order_dev)
    data[key] = {"schedule": list(best.as_tuple()), "times_ms": [float(t) for t in times]}
    store(path, data)
    return best, False
