"""CPU oracle of the learned ranking: a small CNN that predicts a post's
visibility index (Definitions: the visible fraction of the receivers within
the ROI) from the terrain patch around it.  Not part of the paper's method --
it only ranks FINDMAX candidates; VIEWSHED and SITE stay exact.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  float64 numpy, written
from the network's definition, sharing nothing with the HIP kernels.

Network (patch of 64 x 64 posts around the post):
  input  P[dy][dx] = bf16( float32(z[clamp(cy+dy-32, cx+dx-32)] - z[cy,cx]) * 2^-8 ),
         dy, dx in [0, 64): elevation differences in units of 256 m (the
         power-of-two scale is exact, so there is one rounding)
  conv1  4x4 stride 4, 1 -> 16 channels, ReLU         -> 16 x 16 x 16  (H1, bf16)
  conv2  3x3 stride 2, 16 -> 16, ReLU                  ->  7 x  7 x 16  (H2, bf16)
  conv3  3x3 stride 2, 16 -> 32, ReLU                  ->  3 x  3 x 32  (H3, float)
  global average pool -> 32, fully connected 32 -> 1, sigmoid
Conv weights are used in bf16, biases and the head in float.  Loss: mean
squared error against the exact visibility index.  With round=False every
rounding is skipped (a smooth function for finite differences).
"""
from __future__ import annotations

import numpy as np

PATCH = 64
HALF = 32
# (name, shape) in the order of the flat parameter vector
PARAM_SHAPES = [
    ("w1", (16, 4, 4)), ("b1", (16,)),
    ("w2", (16, 3, 3, 16)), ("b2", (16,)),
    ("w3", (32, 3, 3, 16)), ("b3", (32,)),
    ("wfc", (32,)), ("bfc", (1,)),
]
NPARAMS = sum(int(np.prod(s)) for _, s in PARAM_SHAPES)


def unflatten(theta):
    out, o = {}, 0
    for name, shp in PARAM_SHAPES:
        n = int(np.prod(shp))
        out[name] = np.asarray(theta[o:o + n], np.float64).reshape(shp)
        o += n
    return out


def flatten(p):
    return np.concatenate([np.asarray(p[name], np.float64).ravel() for name, _ in PARAM_SHAPES])


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64.
    Values are first rounded to float32 (the GPU holds them in float32)."""
    a = np.asarray(x, np.float32)
    b = a.view(np.uint32).astype(np.uint64)
    rounded = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return rounded.astype(np.uint32).view(np.float32).astype(np.float64)


def patches(z, centres, round=True):
    """Input patches (B, 64, 64) for linear post indices `centres`."""
    z = np.asarray(z)
    nr, nc = z.shape
    c = np.asarray(centres, np.int64)
    cy, cx = c // nc, c % nc
    d = np.arange(PATCH) - HALF
    yy = np.clip(cy[:, None] + d[None, :], 0, nr - 1)
    xx = np.clip(cx[:, None] + d[None, :], 0, nc - 1)
    zz = z[yy[:, :, None], xx[:, None, :]].astype(np.int32) - z[cy, cx].astype(np.int32)[:, None, None]
    if round:
        return bf16(zz.astype(np.float32) * np.float32(2.0 ** -8))
    return zz.astype(np.float64) * 2.0 ** -8


def _conv(x, w, b, stride):
    """x (B, H, W, Ci), w (Co, k, k, Ci): valid convolution with stride."""
    B, H, W, Ci = x.shape
    Co, k, _, _ = w.shape
    Ho, Wo = (H - k) // stride + 1, (W - k) // stride + 1
    out = np.zeros((B, Ho, Wo, Co))
    for ky in range(k):
        for kx in range(k):
            xs = x[:, ky:ky + stride * (Ho - 1) + 1:stride, kx:kx + stride * (Wo - 1) + 1:stride, :]
            out += np.einsum("bhwc,oc->bhwo", xs, w[:, ky, kx, :])
    return out + b


def _conv_back(x, w, dout, stride):
    """Gradients of _conv: (dx, dw, db) for upstream gradient dout."""
    B, H, W, Ci = x.shape
    Co, k, _, _ = w.shape
    Ho, Wo = dout.shape[1], dout.shape[2]
    dx = np.zeros_like(x)
    dw = np.zeros_like(w)
    for ky in range(k):
        for kx in range(k):
            sl = (slice(None), slice(ky, ky + stride * (Ho - 1) + 1, stride),
                  slice(kx, kx + stride * (Wo - 1) + 1, stride), slice(None))
            dw[:, ky, kx, :] = np.einsum("bhwo,bhwc->oc", dout, x[sl])
            dx[sl] += np.einsum("bhwo,oc->bhwc", dout, w[:, ky, kx, :])
    return dx, dw, dout.sum(axis=(0, 1, 2))


def forward(theta, P, round=True):
    """Forward pass; returns a dict of activations (all float64)."""
    p = unflatten(theta)
    R = bf16 if round else (lambda v: np.asarray(v, np.float64))
    x0 = P[:, :, :, None]
    w1 = R(p["w1"])[:, :, :, None]
    a1 = _conv(x0, w1, p["b1"], 4)
    h1 = R(np.maximum(a1, 0))
    a2 = _conv(h1, R(p["w2"]), p["b2"], 2)
    h2 = R(np.maximum(a2, 0))
    a3 = _conv(h2, R(p["w3"]), p["b3"], 2)
    h3 = np.maximum(a3, 0)
    g = h3.mean(axis=(1, 2))
    y = g @ p["wfc"] + p["bfc"][0]
    out = 1.0 / (1.0 + np.exp(-y))
    return {"x0": x0, "h1": h1, "h2": h2, "h3": h3, "g": g, "y": y, "p": out}


def loss(theta, P, t, round=True):
    a = forward(theta, P, round)
    return float(np.mean((a["p"] - t) ** 2))


def backward(theta, P, t, round=True, acts=None):
    """Gradient of the mean squared error w.r.t. the flat parameters.  With
    round=True the upstream gradients entering each convolution are rounded
    to bf16, as the MFMA kernels consume them."""
    p = unflatten(theta)
    R = bf16 if round else (lambda v: np.asarray(v, np.float64))
    a = forward(theta, P, round) if acts is None else acts
    B = P.shape[0]
    dy = 2.0 * (a["p"] - t) / B * a["p"] * (1 - a["p"])
    d_wfc = a["g"].T @ dy
    d_bfc = np.array([dy.sum()])
    dg = dy[:, None] * p["wfc"][None, :]
    da3 = R((dg / 9.0)[:, None, None, :] * (a["h3"] > 0))
    dh2, d_w3, d_b3 = _conv_back(a["h2"], R(p["w3"]), da3, 2)
    da2 = R(dh2 * (a["h2"] > 0))
    dh1, d_w2, d_b2 = _conv_back(a["h1"], R(p["w2"]), da2, 2)
    da1 = R(dh1 * (a["h1"] > 0))
    _, d_w1, d_b1 = _conv_back(a["x0"], R(p["w1"])[:, :, :, None], da1, 4)
    grads = {"w1": d_w1[:, :, :, 0], "b1": d_b1, "w2": d_w2, "b2": d_b2, "w3": d_w3,
             "b3": d_b3, "wfc": d_wfc, "bfc": d_bfc}
    return flatten(grads)


def adam(theta, m, v, g, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba) with bias correction; step counts from 1."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(seed=0):
    """He-style initialisation (a float32-representable start point)."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shp in PARAM_SHAPES:
        if name.startswith("b"):
            p[name] = np.zeros(shp)
        else:
            fan_in = int(np.prod(shp[1:])) if len(shp) > 1 else shp[0]
            p[name] = rng.standard_normal(shp) * np.sqrt(2.0 / fan_in)
    return flatten(p).astype(np.float32).astype(np.float64)
