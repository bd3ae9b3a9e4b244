"""Spectral fractional-Brownian-motion terrains (int16 elevation posts).

Recipe: white N(0,1) noise from a seeded generator, real 2-D FFT, amplitude
scaled by |f|^(-beta/2) (so the power spectrum falls as |f|^-beta), DC set to
zero, inverse FFT, then an affine rescale of [min, max] to [0, zmax] rounded
to the nearest integer.  The paper's terrains are DEMs of integer elevation
posts one unit apart; these stand in for its DEM1000 and NASADEM inputs,
which are not used here.

``fbm`` runs on the host (numpy/PCG64; exact and portable for a given numpy);
``fbm_torch`` runs the same recipe with torch on a device for terrains too
large to synthesise quickly on the host (46400^2).  The two give different
terrains for the same seed; every test passes the same array to both the HIP
path and the oracle, so only determinism within a machine matters.
"""
from __future__ import annotations

import hashlib

import numpy as np


def _spectrum_filter(nrows: int, ncols: int, beta: float, xp=np, device=None):
    if xp is np:
        fy = np.fft.fftfreq(nrows)[:, None]
        fx = np.fft.rfftfreq(ncols)[None, :]
        f = np.sqrt(fy * fy + fx * fx)
        f[0, 0] = 1.0
        a = f ** (-beta / 2.0)
        a[0, 0] = 0.0
        return a
    import torch
    fy = torch.fft.fftfreq(nrows, device=device, dtype=torch.float32)[:, None]
    fx = torch.fft.rfftfreq(ncols, device=device, dtype=torch.float32)[None, :]
    f = torch.sqrt(fy * fy + fx * fx)
    f[0, 0] = 1.0
    a = f.pow(-beta / 2.0)
    a[0, 0] = 0.0
    return a


def _rescale_np(h: np.ndarray, zmax: int) -> np.ndarray:
    lo, hi = float(h.min()), float(h.max())
    s = zmax / (hi - lo) if hi > lo else 0.0
    return np.rint((h - lo) * s).astype(np.int16)


def fbm(n: int, beta: float, zmax: int, seed: int, ncols: int | None = None) -> np.ndarray:
    """Host fBm terrain of shape (n, ncols or n), int16 in [0, zmax]."""
    nrows, ncols = n, (n if ncols is None else ncols)
    rng = np.random.Generator(np.random.PCG64(seed))
    w = rng.standard_normal((nrows, ncols), dtype=np.float32)
    spec = np.fft.rfft2(w)
    spec *= _spectrum_filter(nrows, ncols, beta)
    h = np.fft.irfft2(spec, s=(nrows, ncols))
    return _rescale_np(h, zmax)


def fbm_torch(n: int, beta: float, zmax: int, seed: int, device="cuda", ncols: int | None = None):
    """Device fBm terrain (torch int16 tensor on ``device``), same recipe as
    ``fbm`` with torch's generator; used for the 46400^2 workload."""
    import torch
    nrows, ncols = n, (n if ncols is None else ncols)
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    w = torch.randn((nrows, ncols), generator=g, device=device, dtype=torch.float32)
    spec = torch.fft.rfft2(w)
    del w
    spec *= _spectrum_filter(nrows, ncols, beta, xp=None, device=device)
    h = torch.fft.irfft2(spec, s=(nrows, ncols))
    del spec
    lo, hi = h.min(), h.max()
    h.sub_(lo).mul_(zmax / (hi - lo).clamp_min(1e-30))
    z = torch.round(h).to(torch.int16)
    del h
    return z


def terrain_sha256(z) -> str:
    a = np.ascontiguousarray(z)
    return hashlib.sha256(a.tobytes()).hexdigest()
