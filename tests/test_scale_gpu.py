"""Parity at the workloads' full sizes, in the launch configuration the
benchmark uses.

Where the oracle can afford it, every output of the pass is checked against an
independent oracle chain: the oracle's VIX over the whole terrain, its FINDMAX
on its own counts, its viewsheds of its own candidates, and its greedy SITE on
its own bitmaps -- so a wrong bit anywhere fails.  That is the case for the
46400^2 workload (2.15e9 posts, 81,920 candidates, 4096 observers), the
4096^2 ROI-200 batch and the 16384^2 uneven batch.  The paper-scale ROI runs
(32000^2 at R 500 and 1000, 46400^2 at R 1000 and 2000) are checked on sampled
rows, blocks and windows
plus a replay of the whole selection; a reduced R = 1000 terrain gets the full
oracle chain from FINDMAX on.  SITE with intervisibility is checked on the same
windows wherever the plain one is checked against the oracle.  A terrain of
4.6e9 posts checks the VIX streams of post indices (and a seed) above 2^32."""
import sys
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(*a):
    print("[scale]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def S():
    assert torch.cuda.is_available()
    import paper_2006_16783_amd as S
    return S


@pytest.fixture(autouse=True)
def _release_device_memory():
    # each workload holds up to ~200 GB of window bitmaps: hand torch's cached
    # segments back before and after every test, so that a later workload
    # does not carve its terrain out of an earlier one's bitmap segment and
    # then find no room for its own bitmaps
    import gc
    gc.collect()
    torch.cuda.empty_cache()
    yield
    gc.collect()
    torch.cuda.empty_cache()


def _u64(t):
    return t.cpu().numpy().view(np.uint64)


def _oracle_chain(orc, S, z_host, cfg, res, cnt_or=None, t0=None):
    """Checks the pass `res` (run with keep=True) against the oracle from
    FINDMAX on: candidates, every window bitmap, and the selection, gains and
    cumulative viewshed of the oracle's greedy on its own bitmaps.  The
    FINDMAX key is the oracle's VIX (cnt_or) when given, else the device's."""
    from paper_2006_16783_amd import pipeline as P
    nr, nc = z_host.shape
    t0 = time.time() if t0 is None else t0
    key = cnt_or if cnt_or is not None else res.key.cpu().numpy()
    cand = orc.findmax(key, z_host, cfg.grid, cfg.grid, cfg.k)
    cand = cand[cand >= 0]
    assert len(cand) == len(res.candidates) and (cand == res.candidates).all()
    _say("findmax: all", cfg.grid * cfg.grid, "blocks equal", round(time.time() - t0, 1))
    obs = orc.observers(cand % nc, cand // nc, cfg.roi, cfg.h_t, cfg.h_r)
    bm, off = orc.viewshed(z_host, obs)
    assert (off == res.offsets).all()
    got = _u64(res.bitmaps)[:off[-1]]
    bad = np.nonzero(got != bm)[0]
    assert bad.size == 0, ("viewshed words differ", bad[:8])
    _say("viewsheds: all", len(obs), "windows equal", round(time.time() - t0, 1))
    sel, gains, cum, _ = orc.greedy(bm, off, obs, nr, nc, cfg.max_obs,
                                    P.target_cells(cfg.target_frac, nr, nc), lazy=True)
    assert len(sel) == len(res.selected)
    assert (sel == res.selected).all() and (gains == res.gains).all()
    assert (_u64(res.cumulative).reshape(cum.shape) == cum).all()
    _say("site:", len(sel), "selections, gains and cumulative equal", round(time.time() - t0, 1))
    # the same windows sited with intervisibility (every pick after the first
    # seen by an earlier one), on the device and by the oracle
    tgt = P.target_cells(cfg.target_frac, nr, nc)
    isel, igain, inum, icum = S.siting_greedy(res.bitmaps, torch.from_numpy(off).cuda(),
                                              S.observers_to_device(obs), nr, nc, cfg.max_obs,
                                              tgt, intervisible=True)
    m = int(inum.item())
    wsel, wgain, wcum, _ = orc.greedy(bm, off, obs, nr, nc, cfg.max_obs, tgt, lazy=True,
                                      intervisible=True)
    assert m == len(wsel)
    assert (isel[:m].cpu().numpy() == wsel).all() and (igain[:m].cpu().numpy() == wgain).all()
    assert (_u64(icum).reshape(wcum.shape) == wcum).all()
    _say("site with intervisibility:", m, "selections equal, coverage",
         round(int(wgain.sum()) / (nr * nc), 5), round(time.time() - t0, 1))


def _pass_with_full_oracle(S, orc, cfg):
    from paper_2006_16783_amd import pipeline as P
    from synth import fbm_torch
    t0 = time.time()
    z = fbm_torch(cfg.n, cfg.beta, cfg.zmax, cfg.seed, device="cuda")
    res = P.run(z, cfg, keep=True)
    _say(cfg.name, "pass", res.stage_ms, len(res.observers), len(res.selected))
    z_host = z.cpu().numpy()
    del z
    cnt_or = orc.vix(z_host, cfg.roi, cfg.h_t, cfg.h_r, cfg.K, cfg.vix_seed)
    cnt = res.key.cpu().numpy()
    bad = np.argwhere(cnt != cnt_or)
    assert bad.size == 0, ("vix differs at", bad[:8])
    _say("vix: all", cnt.size, "posts equal", round(time.time() - t0, 1))
    del cnt
    _oracle_chain(orc, S, z_host, cfg, res, cnt_or=cnt_or, t0=t0)


@pytest.mark.timeout(900)
def test_full_scale_46400(S, orc):
    # 46400^2 (2.15e9 posts, 0-4000 m), ROI 100, h 10/10, K 10, 64x64 blocks x
    # 20 = 81,920 candidates, SITE to 4096: every output against the oracle
    from paper_2006_16783_amd import pipeline as P
    _pass_with_full_oracle(S, orc, P.CONFIGS["full_46400"])


@pytest.mark.timeout(600)
def test_batched_4096_r200(S, orc):
    # 4096^2 (0-2000 m), ROI 200, VIX with 50 receivers, 50x50 blocks x 4 =
    # 10,000 tentative observers in one persistent launch, SITE to 2000 or 90%
    from paper_2006_16783_amd import pipeline as P
    _pass_with_full_oracle(S, orc, P.CONFIGS["batched_4096"])


@pytest.mark.timeout(600)
def test_uneven_16384_autotuned(S, orc):
    # 16384^2 (exponent 2.2, 0-3000 m); 40,000 candidates with ROI drawn from
    # 50-400 and height from 5-100 m, edge windows forced; autotuned schedule;
    # SITE to 4000.  Every window, and the oracle's greedy on its own bitmaps.
    from synth import fbm_torch, uniform_observers
    n = 16384
    t0 = time.time()
    z = fbm_torch(n, 2.2, 3000, 1, device="cuda")
    obs = uniform_observers(n, n, 40000, 7, roi=(50, 400), height=(5, 100))
    off = S.siting_viewshed_layout(obs, n, n)
    obs_d = S.observers_to_device(obs)
    off_d = torch.from_numpy(off).cuda()
    order_d = torch.from_numpy(S.siting_viewshed_order(obs)).cuda()
    bm = torch.empty(int(off[-1]), dtype=torch.int64, device="cuda")
    best, times = S.siting_autotune(z, obs_d, off_d, 400, bm, order_dev=order_d)
    _say("autotune", best, [round(t, 2) for t in times])
    bm = S.siting_viewshed_batch(z, obs_d, off_d, 400, order_dev=order_d, sched=best, bitmaps=bm)
    sel, gains, nsel, cum = S.siting_greedy(bm, off_d, obs_d, n, n, 4000, n * n)
    m = int(nsel.item())
    z_host = z.cpu().numpy()
    want, woff = orc.viewshed(z_host, obs)
    assert (woff == off).all()
    bad = np.nonzero(_u64(bm)[:off[-1]] != want)[0]
    assert bad.size == 0, ("viewshed words differ", bad[:8])
    _say("uneven: all", len(obs), "windows equal", round(time.time() - t0, 1))
    wsel, wgain, wcum, _ = orc.greedy(want, off, obs, n, n, 4000, n * n, lazy=True)
    assert m == len(wsel)
    assert (sel[:m].cpu().numpy() == wsel).all() and (gains[:m].cpu().numpy() == wgain).all()
    assert (_u64(cum).reshape(wcum.shape) == wcum).all()
    _say("uneven site ok", m, round(time.time() - t0, 1))
    # with intervisibility (windows of uneven size, heights 5-100 m)
    sel, gains, nsel, cum = S.siting_greedy(bm, off_d, obs_d, n, n, 4000, n * n,
                                            intervisible=True)
    m = int(nsel.item())
    wsel, wgain, wcum, _ = orc.greedy(want, off, obs, n, n, 4000, n * n, lazy=True,
                                      intervisible=True)
    assert m == len(wsel)
    assert (sel[:m].cpu().numpy() == wsel).all() and (gains[:m].cpu().numpy() == wgain).all()
    assert (_u64(cum).reshape(wcum.shape) == wcum).all()
    _say("uneven site with intervisibility ok", m, round(time.time() - t0, 1))


def _check_rows(orc, z_host, cnt_h_rows, cfg, rows):
    want = orc.vix_rows(z_host, cfg.roi, cfg.h_t, cfg.h_r, cfg.K, cfg.vix_seed, rows)
    bad = np.argwhere(cnt_h_rows != want)
    assert bad.size == 0, ("vix rows differ", [(rows[i], j) for i, j in bad[:8]])


def _check_blocks(orc, cnt_h, z_host, cand, G, k):
    want = orc.findmax(cnt_h, z_host, G, G, k)
    assert (cand == want[want >= 0]).all()


def _edge_picks(obs, nr, nc, n, rng):
    R = obs["roi"].astype(np.int64)
    edge = np.nonzero((obs["x"] < R) | (obs["y"] < R) | (obs["x"] >= nc - R) | (obs["y"] >= nr - R))[0]
    picks = list(edge[:n // 4]) + list(rng.choice(len(obs), n - min(len(edge), n // 4), replace=False))
    return sorted(set(int(p) for p in picks))


def _paper_roi_pass(S, orc, name, n_views):
    """A paper-scale ROI configuration: VIX rows (1 in 500 and the edges),
    every FINDMAX block from the device counts, sampled viewsheds (edge windows
    included) against the oracle, the first pick against the largest
    viewshed, and a replay of every selection over the device bitmaps."""
    from paper_2006_16783_amd import pipeline as P
    from synth import fbm_torch
    cfg = P.CONFIGS[name]
    t0 = time.time()
    z = fbm_torch(cfg.n, cfg.beta, cfg.zmax, cfg.seed, device="cuda")
    res = P.run(z, cfg, keep=True)
    _say(name, "pass", res.stage_ms, len(res.observers), len(res.selected))
    assert len(res.observers) == cfg.grid * cfg.grid * cfg.k
    assert 0 < len(res.selected) <= cfg.max_obs
    z_host = z.cpu().numpy()
    rows = sorted(set([0, 1, cfg.n - 2, cfg.n - 1] + list(range(7, cfg.n, 500))))
    _check_rows(orc, z_host, res.key[rows].cpu().numpy(), cfg, rows)
    _say("vix rows ok", len(rows), round(time.time() - t0, 1))
    _check_blocks(orc, res.key.cpu().numpy(), z_host, res.candidates, cfg.grid, cfg.k)
    _say("findmax: all blocks ok", round(time.time() - t0, 1))
    obs, off = res.observers, res.offsets
    picks = _edge_picks(obs, cfg.n, cfg.n, n_views, np.random.default_rng(5))

    def window(i):  # one window's words, copied from the device
        return _u64(res.bitmaps[int(off[i]):int(off[i + 1])])

    for i in picks:
        one = orc.viewshed_one(z_host, obs[i]).ravel()
        assert (window(i) == one).all(), ("viewshed", i, obs[i])
    _say("viewsheds ok", len(picks), round(time.time() - t0, 1))
    # SITE: the first pick is the largest viewshed (ties to the lowest index;
    # visible counts from the count sink), and replaying the selection over
    # the device bitmaps gives every recorded gain
    # (above ROI 1087 the count sink rebuilds each window in the bitmaps it
    # is given: the pass's own, rewritten with the same bits)
    vis, _ = S.siting_viewshed_batch(z, S.observers_to_device(obs), torch.from_numpy(off).cuda(),
                                     cfg.roi, sink=S.SITING_SINK_COUNT, bitmaps=res.bitmaps)
    vis = vis.cpu().numpy().astype(np.int64)
    assert res.selected[0] == int(np.argmax(vis)) and res.gains[0] == vis.max()
    W = (cfg.n + 63) // 64
    C = np.zeros((cfg.n, W), np.uint64)
    for t, i in enumerate(res.selected):
        o = obs[i]
        R, x, y = int(o["roi"]), int(o["x"]), int(o["y"])
        ylo, yhi = max(0, y - R), min(cfg.n - 1, y + R)
        w0, w1 = max(0, x - R) >> 6, min(cfg.n - 1, x + R) >> 6
        win = window(i).reshape(yhi - ylo + 1, w1 - w0 + 1)
        cv = C[ylo:yhi + 1, w0:w1 + 1]
        g = int(np.bitwise_count(win & ~cv).sum())
        assert g == res.gains[t], ("site replay", t, i, g, res.gains[t])
        cv |= win
    assert (np.diff(res.gains) <= 0).all()
    assert (_u64(res.cumulative).reshape(C.shape) == C).all()
    _say(name, "site replay ok", round(time.time() - t0, 1))


@pytest.mark.timeout(900)
def test_paper_roi_east_32000_r1000(S, orc):
    # the paper's second billion-post run as a synthetic stand-in: 32000^2,
    # ROI 1000 (quadrant-mode viewsheds), h 100/10, 96x96 blocks x 20 =
    # 184,320 candidates, SITE to 5000 (four-wavefront rounds)
    _paper_roi_pass(S, orc, "east_32000_r1000", 24)


@pytest.mark.timeout(900)
def test_paper_roi_east_32000_r500(S, orc):
    # the paper's first billion-post run: 32000^2, ROI 500, h 100/10,
    # 193x193 blocks x 20 = 744,980 candidates, SITE to 6543
    _paper_roi_pass(S, orc, "east_32000_r500", 48)


@pytest.mark.timeout(900)
def test_paper_roi_west_46400_r1000(S, orc):
    # the paper's first US-West run: 46400^2 (0-2706 m), ROI 1000, h 100/10,
    # 139x139 blocks x 20 = 386,420 candidates, SITE to 5647
    _paper_roi_pass(S, orc, "west_46400_r1000", 24)


@pytest.mark.timeout(900)
def test_paper_roi_west_46400_r2000(S, orc):
    # the paper's second US-West run: ROI 2000 (global-bitmap viewsheds),
    # 70x70 blocks x 20 = 98,000 candidates, SITE to 3347
    _paper_roi_pass(S, orc, "west_46400_r2000", 16)


@pytest.mark.timeout(600)
def test_reduced_r1000_full_oracle(S, orc):
    # ROI 1000 on a 4096^2 terrain (0-507 m, h 100/10): the paper's block rule
    # (round(4096 / 333) = 12 per side), 4 per block = 576 candidates, every
    # window (quadrant mode, clipped on every side) and the whole selection
    # against the oracle's chain from FINDMAX on
    from paper_2006_16783_amd import pipeline as P
    from synth import fbm_torch
    cfg = P.SitingConfig("reduced_4096_r1000", 4096, 2.4, 507, 3, 1000, 100, 10, 10, 12, 4,
                         300, 1.0)
    t0 = time.time()
    z = fbm_torch(cfg.n, cfg.beta, cfg.zmax, cfg.seed, device="cuda")
    res = P.run(z, cfg, keep=True)
    _say("reduced r1000 pass", res.stage_ms, len(res.observers), len(res.selected))
    z_host = z.cpu().numpy()
    rows = [0, 1, 1000, 2047, 3000, 4094, 4095]
    _check_rows(orc, z_host, res.key[rows].cpu().numpy(), cfg, rows)
    _oracle_chain(orc, S, z_host, cfg, res, t0=t0)


@pytest.mark.timeout(600)
def test_vix_post_index_and_seed_above_2_32(S, orc):
    # 320 x 14,401,536 posts (4.6e9): rows from 299 on hold post indices
    # >= 2^32 (row 298 straddles it), so the stream's counter word 2 (t / 2^32)
    # is non-zero there; the seed is above 2^32 too (key word 1 non-zero)
    from synth import fbm
    nr, tile, reps = 320, 4096, 3516
    nc = tile * reps
    assert nr * nc > 2 ** 32 and 298 * nc < 2 ** 32 < 299 * nc
    R, K, seed = 3, 10, (5 << 32) | 99
    base = torch.from_numpy(fbm(nr, 2.4, 900, 9, ncols=tile)).cuda()
    z = base.repeat(1, reps)
    del base
    cnt = S.siting_vix(z, R, 10, 10, K, seed)
    rows = [0, 1, 298, 299, 310, 318, 319]
    got = cnt[rows].cpu().numpy()
    del cnt
    # the oracle's terrain: only the rows the checked lines of sight can read
    # hold data (the rest of the array is never touched)
    z_host = np.zeros((nr, nc), np.int16)
    for r0, r1 in [(0, 5), (295, nr)]:
        z_host[r0:r1] = z[r0:r1].cpu().numpy()
    del z
    want = orc.vix_rows(z_host, R, 10, 10, K, seed, rows)
    bad = np.argwhere(got != want)
    assert bad.size == 0, ("vix differs", [(rows[i], j) for i, j in bad[:8]])
    _say("vix rows above 2^32 ok", rows)
