"""Pins of the CNN oracle: float64 gradients against central finite
differences, the convolution against a direct loop definition, bf16
rounding against exhaustive bit-level rules, and Adam against its first-step
closed form."""
import numpy as np
import pytest

from oracle import cnn
from synth import fbm


def _setup(B=3, seed=0):
    z = fbm(120, 2.4, 900, 5 + seed)
    rng = np.random.default_rng(seed)
    centres = rng.integers(0, 120 * 120, size=B)
    centres[0] = 0          # corner: clamped patch
    P = cnn.patches(z, centres, round=False)
    t = rng.random(B)
    theta = cnn.init_params(seed)
    return z, centres, P, t, theta


def test_gradient_matches_finite_differences():
    _, _, P, t, theta = _setup()
    g = cnn.backward(theta, P, t, round=False)
    rng = np.random.default_rng(1)
    idx = np.concatenate([rng.choice(cnn.NPARAMS, 40, replace=False), [cnn.NPARAMS - 1]])
    h = 1e-5
    for i in idx:
        e = np.zeros_like(theta)
        e[i] = h
        fd = (cnn.loss(theta + e, P, t, False) - cnn.loss(theta - e, P, t, False)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-8, np.abs(g).max()) + 1e-6 * abs(fd), (i, fd, g[i])


def test_conv_matches_loop_definition():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, 9, 11, 3))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    out = cnn._conv(x, w, b, 2)
    for bb in range(2):
        for oy in range(out.shape[1]):
            for ox in range(out.shape[2]):
                for o in range(4):
                    s = b[o]
                    for ky in range(3):
                        for kx in range(3):
                            for c in range(3):
                                s += w[o, ky, kx, c] * x[bb, 2 * oy + ky, 2 * ox + kx, c]
                    assert abs(out[bb, oy, ox, o] - s) < 1e-12


def test_bf16_rounding_rules():
    # exactly representable values stay; halfway cases go to even mantissas
    vals = np.array([1.0, -2.5, 0.0, 2.0 ** 100, -0.375], np.float32)
    assert (cnn.bf16(vals) == vals.astype(np.float64)).all()
    one = np.float32(1.0).view(np.uint32)
    half_ulp = np.uint32(one + 0x8000).view(np.float32)       # 1 + 2^-8 -> ties to 1.0
    assert cnn.bf16(half_ulp) == 1.0
    odd = np.uint32(one + 0x10000).view(np.float32)             # 1 + 2^-7 (odd mantissa)
    tie_up = np.uint32(one + 0x18000).view(np.float32)
    assert cnn.bf16(tie_up) == float(np.uint32(one + 0x20000).view(np.float32))
    assert cnn.bf16(odd) == float(odd)
    just_above = np.uint32(one + 0x8001).view(np.float32)
    assert cnn.bf16(just_above) == float(odd)


def test_patch_centre_and_clamp():
    z = np.arange(100 * 90, dtype=np.int64).reshape(100, 90).astype(np.int16)
    P = cnn.patches(z, [0, 50 * 90 + 45], round=False)
    assert P.shape == (2, 64, 64)
    assert P[0, 32, 32] == 0 and P[1, 32, 32] == 0
    # clamped corner: the rows above the terrain repeat row 0
    assert (P[0, :32, 32] == 0).all()
    assert P[1, 33, 32] == 90 / 256 and P[1, 32, 33] == 1 / 256
    assert P[1, 0, 0] == (-32 * 90 - 32) / 256


def test_adam_constant_gradient_moves_lr_per_step():
    # with a constant gradient g the bias-corrected moments are exactly g and
    # g^2 at every step (m_t = (1 - b1^t) g, v_t = (1 - b2^t) g^2), so every
    # step moves each parameter by lr * g / (|g| + eps): the bias correction
    # of Adam (Kingma & Ba, Algorithm 1) pinned at steps 1..50, not just the first
    rng = np.random.default_rng(5)
    theta0 = rng.standard_normal(12)
    g = rng.standard_normal(12) * np.logspace(-3, 2, 12)
    lr, eps = 0.003, 1e-8
    theta, m, v = theta0.copy(), np.zeros(12), np.zeros(12)
    for step in range(1, 51):
        prev = theta
        theta, m, v = cnn.adam(theta, m, v, g, step, lr, eps=eps)
        assert np.allclose(prev - theta, lr * g / (np.abs(g) + eps), rtol=1e-9, atol=1e-15), step
    assert np.allclose(theta, theta0 - 50 * lr * g / (np.abs(g) + eps), rtol=0, atol=1e-12)
    assert np.allclose(theta, theta0 - 50 * lr * np.sign(g), rtol=0, atol=1e-5)


def test_adam_first_step_is_signed_lr():
    rng = np.random.default_rng(3)
    theta = rng.standard_normal(10)
    g = rng.standard_normal(10)
    new, m, v = cnn.adam(theta, np.zeros(10), np.zeros(10), g, 1, 0.01)
    assert np.allclose(new, theta - 0.01 * np.sign(g), atol=1e-6)


def test_rounded_forward_close_to_exact():
    _, _, P, t, theta = _setup(B=4)
    Pr = cnn.bf16(P)
    a = cnn.forward(theta, Pr, round=True)["p"]
    b = cnn.forward(theta, P, round=False)["p"]
    assert np.allclose(a, b, atol=2e-2)
