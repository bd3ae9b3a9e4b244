"""The CNN kernels (BF16 MFMA, FP32 accumulation) against the float64 oracle on
the same inputs.

Tolerances: the oracle rounds to bf16 at the points the kernels do, but it
rounds float64 sums while the kernels round float32 sums, so an activation
lying within float32 error of a bf16 rounding boundary can land one bf16 ulp
(2^-8 relative) apart.  Such flips are rare and their effect on the outputs is
bounded by (weights x 2^-8 x the activation), which gives the tolerances
below (an order of magnitude above the observed spread, far below any real
error: a wrong weight index or layout moves outputs by O(1)).  Gradients are
compared element by element against a bound derived in that test."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def S():
    assert torch.cuda.is_available()
    import paper_2006_16783_amd as S
    return S


def _case(seed, B, n=300):
    from synth import fbm
    from oracle import cnn
    z = fbm(n, 2.4, 2000, seed)
    rng = np.random.default_rng(seed)
    centres = rng.integers(0, n * n, size=B)
    centres[:4] = [0, n - 1, n * n - 1, (n // 2) * n + n // 2]
    theta = cnn.init_params(seed).astype(np.float32)
    labels = rng.random(B).astype(np.float32)
    return z, centres, theta, labels


def _dev(a, dt=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    return (t if dt is None else t.to(dt)).cuda()


def test_forward_matches_oracle(S):
    from oracle import cnn
    z, centres, theta, _ = _case(1, 96)
    ws = S.cnn_workspace(96)
    pred = S.siting_cnn_forward(_dev(theta), _dev(z), _dev(centres.astype(np.int64)), ws)
    P = cnn.patches(z, centres, round=True)
    want = cnn.forward(theta.astype(np.float64), P, round=True)["p"]
    got = pred.cpu().numpy()
    print("max |dp|", np.abs(got - want).max(), flush=True)
    assert np.abs(got - want).max() < 2e-3


def test_score_equals_forward_at_cell_maxima(S):
    from oracle import cnn
    from synth import fbm
    z = fbm(170, 2.2, 1500, 3, ncols=203)
    theta = cnn.init_params(3).astype(np.float32)
    import oracle
    for stride in (4, 7, 1, 8):
        sc = S.siting_cnn_score_terrain(_dev(theta), _dev(z), stride).cpu().numpy()
        # each cell is scored at its highest post
        centres = oracle.cell_max(z, stride)
        ws = S.cnn_workspace(len(centres))
        pred = S.siting_cnn_forward(_dev(theta), _dev(z), _dev(centres), ws).cpu().numpy()
        # same arithmetic in the same order: identical bits
        assert (pred == sc.ravel()).all(), stride
        P = cnn.patches(z, centres, round=True)
        want = cnn.forward(theta.astype(np.float64), P, round=True)["p"]
        assert np.abs(pred - want).max() < 2e-3


@pytest.mark.parametrize("n,ncols,stride,zlo,zhi", [
    (1600, 1600, 8, 0, 3000),      # dword staging, two tiles per workgroup
    (1040, 1040, 4, 0, 3000),      # 16 x 16 cells per tile
    (300, 256, 8, -30000, 30000),  # elevation range above 32767
    (300, 256, 5, -30000, 30000),
])
def test_score_paths_equal_forward(S, n, ncols, stride, zlo, zhi):
    """Scoring's tile staging (dword moves on interior tiles of an even-pitch
    terrain, post by post at the edges), its 16-bit differences (tiles whose
    elevation range fits 16 bits) and its runs of tiles per workgroup give the
    training forward's bits at every cell maximum; a sample against the
    oracle where the range is realistic."""
    from oracle import cnn
    from synth import fbm
    import oracle
    z = fbm(n, 2.2, 3000, 11, ncols=ncols).astype(np.int64)
    z = (zlo + (z - z.min()) * (zhi - zlo) // max(1, int(z.max() - z.min()))).astype(np.int16)
    theta = cnn.init_params(5).astype(np.float32)
    sc = S.siting_cnn_score_terrain(_dev(theta), _dev(z), stride).cpu().numpy().ravel()
    centres = oracle.cell_max(z, stride)
    ws = S.cnn_workspace(len(centres))
    pred = S.siting_cnn_forward(_dev(theta), _dev(z), _dev(centres), ws).cpu().numpy()
    del ws
    assert (pred == sc).all(), int((pred != sc).sum())
    if zhi - zlo <= 3000:
        pick = np.random.default_rng(n).choice(len(centres), 48, replace=False)
        P = cnn.patches(z, centres[pick], round=True)
        want = cnn.forward(theta.astype(np.float64), P, round=True)["p"]
        assert np.abs(sc[pick] - want).max() < 2e-3


def test_backward_matches_oracle(S):
    from oracle import cnn
    z, centres, theta, labels = _case(2, 200)
    ws = S.cnn_workspace(200)
    th = _dev(theta)
    S.siting_cnn_forward(th, _dev(z), _dev(centres.astype(np.int64)), ws)
    grad, loss = S.siting_cnn_backward(th, _dev(labels), ws)
    got = grad.cpu().numpy().astype(np.float64)
    P = cnn.patches(z, centres, round=True)
    t64 = theta.astype(np.float64)
    want = cnn.backward(t64, P, labels.astype(np.float64), round=True)
    want_loss = cnn.loss(t64, P, labels.astype(np.float64), round=True)
    got_loss = float(loss.cpu()[0])
    assert abs(got_loss - want_loss) <= 1e-4 * abs(want_loss) + 1e-7, (got_loss, want_loss)
    # element by element, per parameter tensor: |g - w| <= 1e-3 |w| + atol with
    # atol = 2^-8 x rms(w) -- a bf16 flip of one activation moves a gradient
    # element by at most one of its terms x 2^-7, far below the tensor's rms
    # (float32 summation order adds ~1e-5 relative); a wrong bias, channel or
    # tap moves its elements by O(|w|)
    off = 0
    for name, shp in cnn.PARAM_SHAPES:
        n = int(np.prod(shp))
        g, w = got[off:off + n], want[off:off + n]
        atol = 2.0 ** -8 * float(np.sqrt(np.mean(w * w)))
        bound = 1e-3 * np.abs(w) + atol
        worst = float((np.abs(g - w) / bound).max())
        print(name, "worst |g-w| / bound", worst, "atol", atol, flush=True)
        assert (np.abs(g - w) <= bound).all(), (name, np.argmax(np.abs(g - w) / bound))
        off += n


def test_adam_matches_oracle(S):
    from oracle import cnn
    rng = np.random.default_rng(4)
    n = cnn.NPARAMS
    theta = rng.standard_normal(n).astype(np.float32)
    m = np.zeros(n, np.float32)
    v = np.zeros(n, np.float32)
    tp, tm, tv = _dev(theta), _dev(m), _dev(v)
    t64, m64, v64 = theta.astype(np.float64), m.astype(np.float64), v.astype(np.float64)
    for step in range(1, 4):
        g = rng.standard_normal(n).astype(np.float32)
        S.siting_cnn_adam(tp, tm, tv, _dev(g), step, 1e-3)
        t64, m64, v64 = cnn.adam(t64, m64, v64, g.astype(np.float64), step, 1e-3)
    assert np.allclose(tp.cpu().numpy(), t64, rtol=1e-5, atol=1e-6)


def test_training_reduces_loss(S):
    from oracle import cnn
    z, centres, theta, labels = _case(5, 256)
    # a learnable target: the centre's relative height in its patch
    P = cnn.patches(z, centres, round=False)
    labels = (1.0 / (1.0 + np.exp(-P.mean(axis=(1, 2)) * 256.0 / 200.0))).astype(np.float32)
    ws = S.cnn_workspace(256)
    th, m, v = _dev(theta), torch.zeros(cnn.NPARAMS, device="cuda"), torch.zeros(cnn.NPARAMS, device="cuda")
    zd, cd, ld = _dev(z), _dev(centres.astype(np.int64)), _dev(labels)
    losses = []
    for step in range(1, 81):
        S.siting_cnn_forward(th, zd, cd, ws)
        g, loss = S.siting_cnn_backward(th, ld, ws)
        losses.append(float(loss.cpu()[0]))
        S.siting_cnn_adam(th, m, v, g, step, 1e-3)
    print("loss", losses[0], losses[-1], flush=True)
    assert losses[-1] < 0.2 * losses[0]
