"""Parity of the HIP path (through the C ABI) with the CPU oracle: bit-exact
on seeded fBm terrains, at sizes that span several tiles with ragged tails,
clipped edge windows and uneven ROIs."""
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def S():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2006_16783_amd as S
    return S


def _terrain(n, beta, zmax, seed, ncols=None):
    from synth import fbm
    return fbm(n, beta, zmax, seed, ncols=ncols)


def _u64(t):
    return t.cpu().numpy().view(np.uint64)


# ---------------------------------------------------------------- VIX ------
@pytest.mark.parametrize("shape,R,ht,hr,K,seed", [
    ((300, 257), 20, 10, 10, 10, 1),     # LDS tiles with ragged edges
    ((130, 517), 7, 0, 0, 255, 99),      # K at its maximum, zero heights
    ((64, 64), 100, 10, 10, 10, 5),      # ROI larger than the terrain
    ((421, 380), 140, 25, 3, 6, 7),      # too big for an LDS tile: global reads
    ((520, 610), 30, 5, 15, 23, 11),     # several chunks and batches per wavefront
    ((257, 301), 12, 10, 10, 10, (3 << 32) | 17),  # seed above 2^32: key word 1 non-zero
])
def test_vix_parity(S, orc, shape, R, ht, hr, K, seed):
    _say("vix", shape, R, ht, hr, K, seed)
    z = _terrain(shape[0], 2.4, 1500, seed % 1000, ncols=shape[1])
    zd = torch.from_numpy(z).cuda()
    vseed = seed * 7919 if seed < 2 ** 32 else seed
    got = S.siting_vix(zd, R, ht, hr, K, vseed).cpu().numpy()
    want = orc.vix(z, R, ht, hr, K, vseed)
    assert (got == want).all(), int((got != want).sum())


@pytest.mark.parametrize("shape,ld,R", [((300, 310), 310, 140), ((257, 200), 203, 150)])
def test_vix_global_reads_stay_in_the_terrain(S, orc, shape, ld, R):
    # ROI above the largest LDS tile: the kernel reads the terrain through the
    # cache hierarchy.  Lines of sight along a row or column end at posts of
    # the last row or column; the counting variant records the lowest and
    # highest element offset it reads, which must stay in the terrain (the
    # allocation is exactly nrows * ld - (ld - ncols) posts long).
    nr, nc = shape
    z = _terrain(nr, 2.4, 900, 17, ncols=nc)
    flat = torch.zeros(nr * ld - (ld - nc), dtype=torch.int16, device="cuda")
    view = torch.as_strided(flat, (nr, nc), (ld, 1))
    view.copy_(torch.from_numpy(z).cuda())
    cnt, steps, tests, (lo, hi) = S.siting_vix_stats(view, R, 10, 10, 12, 5)
    _say("vix global reads", shape, ld, R, lo, hi, steps, tests)
    assert 0 <= lo <= hi <= (nr - 1) * ld + nc - 1, (lo, hi)
    assert lo == 0 and hi == (nr - 1) * ld + nc - 1   # the corners are read (own posts)
    assert (cnt.cpu().numpy() == orc.vix(z, R, 10, 10, 12, 5)).all()
    assert (S.siting_vix(view, R, 10, 10, 12, 5).cpu().numpy() == cnt.cpu().numpy()).all()


def test_vix_lds_tile_reads_stay_in_the_terrain(S):
    # the LDS-tiled path reads the terrain only while staging tiles
    z = _terrain(300, 2.4, 900, 18, ncols=262)
    zd = torch.from_numpy(z).cuda()
    _, _, _, (lo, hi) = S.siting_vix_stats(zd, 30, 10, 10, 10, 5)
    assert lo == 0 and hi == 300 * 262 - 1


def test_vix_strided_terrain(S, orc):
    z = _terrain(200, 2.2, 800, 3, ncols=300)
    big = torch.zeros((200, 320), dtype=torch.int16, device="cuda")
    big[:, :300] = torch.from_numpy(z).cuda()
    got = S.siting_vix(big[:, :300], 15, 5, 5, 9, 4).cpu().numpy()
    assert (got == orc.vix(z, 15, 5, 5, 9, 4)).all()


# ------------------------------------------------------------ FINDMAX ------
@pytest.mark.parametrize("shape,g_r,g_c,k", [((1000, 1000), 10, 10, 10), ((333, 517), 7, 3, 20),
                                            ((97, 101), 97, 101, 1), ((250, 250), 4, 4, 32),
                                            # 16-aligned rows (16-byte streaming), ragged blocks
                                            ((480, 512), 7, 9, 20), ((130, 1024), 3, 5, 3),
                                            ((64, 4096), 2, 3, 32)])
def test_findmax_u8_parity(S, orc, shape, g_r, g_c, k):
    _say("findmax", shape, g_r, g_c, k)
    rng = np.random.default_rng(k)
    z = _terrain(shape[0], 2.4, 500, 11, ncols=shape[1])
    key = rng.integers(0, 11, size=shape).astype(np.uint8)
    got = S.siting_findmax(torch.from_numpy(key).cuda(), torch.from_numpy(z).cuda(), g_r, g_c,
                           k).cpu().numpy()
    assert (got == orc.findmax(key, z, g_r, g_c, k)).all()


@pytest.mark.parametrize("stride", [1, 3, 4])
def test_findmax_f32_parity(S, orc, stride):
    z = _terrain(410, 2.4, 500, 12, ncols=390)
    kr, kc = -(-410 // stride), -(-390 // stride)
    rng = np.random.default_rng(stride)
    sc = rng.random((kr, kc), dtype=np.float32)
    sc[rng.random((kr, kc)) < 0.05] = 0.5            # ties
    sc[0, :7] = np.nan
    sc[1, :3] = -np.inf
    got = S.siting_findmax(torch.from_numpy(sc).cuda(), torch.from_numpy(z).cuda(), 9, 8, 20,
                           key_stride=stride).cpu().numpy()
    assert (got == orc.findmax(sc, z, 9, 8, 20, stride=stride)).all()


# ----------------------------------------------------------- VIEWSHED ------
def _viewshed_case(S, orc, z, obs, rmax, sched=None):
    nr, nc = z.shape
    zd = torch.from_numpy(z).cuda()
    off = S.siting_viewshed_layout(obs, nr, nc)
    obs_d = S.observers_to_device(obs)
    off_d = torch.from_numpy(off).cuda()
    order_d = torch.from_numpy(S.siting_viewshed_order(obs)).cuda()
    bm = S.siting_viewshed_batch(zd, obs_d, off_d, rmax, order_dev=order_d, sched=sched)
    want, woff = orc.viewshed(z, obs)
    assert (woff == off).all()
    return _u64(bm)[:off[-1]], want


def test_viewshed_plain_1000_candidates(S, orc):
    # the plain workload: 1000^2, ROI 100, h = 10/10, 1000 candidates
    z = _terrain(1000, 2.4, 1000, 1)
    from synth import uniform_observers
    obs = uniform_observers(1000, 1000, 1000, 5, roi=(100, 100), height=(10, 10))
    got, want = _viewshed_case(S, orc, z, obs, 100)
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, bad[:10]


@pytest.mark.parametrize("seed,roi,height,shape", [
    (1, (1, 40), (0, 30), (300, 350)),
    (2, (50, 160), (5, 100), (700, 640)),
    (3, (150, 300), (0, 200), (650, 701)),
    (4, (300, 450), (0, 60), (1000, 980)),   # one workgroup of 16 wavefronts per CU
])
def test_viewshed_uneven_clipped(S, orc, seed, roi, height, shape):
    _say("viewshed uneven", seed, roi, shape)
    from synth import uniform_observers
    z = _terrain(shape[0], 2.2, 3000, seed, ncols=shape[1])
    obs = uniform_observers(shape[0], shape[1], 300, seed, roi=roi, height=height)
    got, want = _viewshed_case(S, orc, z, obs, roi[1])
    assert (got == want).all()


@pytest.mark.parametrize("ld", [340, 341])
def test_viewshed_strided_terrain(S, orc, ld):
    # a 300x330 terrain inside wider rows: an even leading dimension stages the
    # quadrants straight from HBM into LDS, an odd one through registers
    _say("viewshed strided", ld)
    z = _terrain(300, 2.4, 1500, 13, ncols=330)
    big = torch.zeros((300, ld), dtype=torch.int16, device="cuda")
    big[:, :330] = torch.from_numpy(z).cuda()
    from synth import uniform_observers
    obs = uniform_observers(300, 330, 120, 13, roi=(10, 90), height=(0, 40))
    off = S.siting_viewshed_layout(obs, 300, 330)
    bm = S.siting_viewshed_batch(big[:, :330], S.observers_to_device(obs),
                                 torch.from_numpy(off).cuda(), 90)
    want, _ = orc.viewshed(z, obs)
    assert (_u64(bm)[:off[-1]] == want).all()


def _quadrant_observers(nr, nc, n, seed, roi, height):
    # uniform posts plus the four corners and the four edge midpoints
    from synth import uniform_observers
    obs = uniform_observers(nr, nc, n, seed, roi=roi, height=height)
    ex = np.zeros(8, obs.dtype)
    ex["x"] = [0, nc - 1, 0, nc - 1, nc // 2, nc // 2, 0, nc - 1]
    ex["y"] = [0, 0, nr - 1, nr - 1, 0, nr - 1, nr // 2, nr // 2]
    ex["roi"], ex["h_t"], ex["h_r"] = roi[1], height[1], height[0]
    return np.concatenate([obs, ex])


@pytest.mark.parametrize("seed,roi,shape", [
    (31, (560, 800), (1300, 1250)),   # every window in quadrant mode
    (32, (5, 700), (1100, 1170)),     # small and large ROIs in one quadrant-mode batch
])
def test_viewshed_quadrant_mode(S, orc, seed, roi, shape):
    # windows whose bitmap exceeds LDS: one quadrant at a time, both sinks
    _say("viewshed quadrant mode", seed, roi, shape)
    nr, nc = shape
    z = _terrain(nr, 2.4, 2500, seed, ncols=nc)
    obs = _quadrant_observers(nr, nc, 40, seed, roi, (0, 60))
    got, want = _viewshed_case(S, orc, z, obs, roi[1])
    assert (got == want).all()
    vis, cells = S.siting_viewshed_batch(torch.from_numpy(z).cuda(), S.observers_to_device(obs),
                                         None, roi[1], sink=S.SITING_SINK_COUNT)
    wv, wc = orc.viewshed_count(z, obs)
    assert (vis.cpu().numpy().astype(np.uint32) == wv).all()
    assert (cells.cpu().numpy().astype(np.uint32) == wc).all()


@pytest.mark.timeout(600)
def test_viewshed_global_bitmap_mode(S, orc):
    # ROI 1100-2000 (the paper's second US-West run uses 2000): a quadrant's
    # bitmap exceeds LDS, so each window is cleared and marked in HBM.  A
    # 4600^2 terrain (so R = 2000 windows are clipped on one side or more),
    # the corners and edge midpoints included, every window against the
    # oracle; then SITE on those windows against the oracle's greedy
    seed, nr, nc, roi = 71, 4600, 4600, (1100, 2000)
    _say("viewshed global-bitmap mode", seed, nr, nc, roi)
    z = _terrain(nr, 2.4, 2700, seed, ncols=nc)
    obs = _quadrant_observers(nr, nc, 24, seed, roi, (5, 100))
    got, want = _viewshed_case(S, orc, z, obs, roi[1])
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, ("viewshed words differ", bad[:8])
    _say("windows equal", len(obs))
    # the count sink builds the windows in the caller's bitmaps (required here)
    off = S.siting_viewshed_layout(obs, nr, nc)
    zd, obs_d, off_d = torch.from_numpy(z).cuda(), S.observers_to_device(obs), torch.from_numpy(off).cuda()
    with pytest.raises(S.SitingError) as ei:
        S.siting_viewshed_batch(zd, obs_d, None, roi[1], sink=S.SITING_SINK_COUNT)
    assert ei.value.code == -1
    scratch = torch.empty(int(off[-1]), dtype=torch.int64, device="cuda")
    vis, cells = S.siting_viewshed_batch(zd, obs_d, off_d, roi[1], sink=S.SITING_SINK_COUNT,
                                         bitmaps=scratch)
    wv, wc = orc.viewshed_count(z, obs)
    assert (vis.cpu().numpy().astype(np.uint32) == wv).all()
    assert (cells.cpu().numpy().astype(np.uint32) == wc).all()
    assert (_u64(scratch) == want).all()
    wsel, wgain, wcum, _ = orc.greedy(want, off, obs, nr, nc, 20, nr * nc, lazy=True)
    bm = torch.from_numpy(want.view(np.int64)).cuda()
    sel, gains, nsel, cum = S.siting_greedy(bm, torch.from_numpy(off).cuda(),
                                            S.observers_to_device(obs), nr, nc, 20, nr * nc)
    m = int(nsel.item())
    assert m == len(wsel) and (sel[:m].cpu().numpy() == wsel).all()
    assert (gains[:m].cpu().numpy() == wgain).all()
    assert (_u64(cum).reshape(-1) == wcum.reshape(-1)).all()


@pytest.mark.parametrize("seed,roi,height,shape", [
    (41, (1, 40), (0, 30), (200, 230)),
    (42, (30, 90), (5, 100), (300, 280)),
])
def test_viewshed_r3_exact(S, orc, seed, roi, height, shape):
    # exact per-cell viewsheds, edge windows and the corners included
    _say("viewshed r3", seed, roi, shape)
    nr, nc = shape
    z = _terrain(nr, 2.3, 1200, seed, ncols=nc)
    obs = _quadrant_observers(nr, nc, 60, seed, roi, height)
    off = S.siting_viewshed_layout(obs, nr, nc)
    got = S.siting_viewshed_r3(torch.from_numpy(z).cuda(), S.observers_to_device(obs),
                               torch.from_numpy(off).cuda())
    want, woff = orc.viewshed_r3(z, obs)
    assert (woff == off).all()
    assert (_u64(got)[:off[-1]] == want).all()


def test_viewshed_every_schedule_same_bits(S, orc):
    from synth import uniform_observers
    z = _terrain(500, 2.4, 2000, 8)
    obs = uniform_observers(500, 500, 200, 8, roi=(30, 120), height=(2, 40))
    want, _ = orc.viewshed(z, obs)
    for sc in S.siting_autotune_candidates(120):
        _say("schedule", sc)
        got, _ = _viewshed_case(S, orc, z, obs, 120, sched=sc)
        assert (got == want).all(), sc


@pytest.mark.parametrize("seed,roi,shape,relief", [
    (91, (150, 400), (900, 870), 2000),      # terrain read from global memory, bitmap in LDS
    (92, (60, 120), (260, 270), None),       # extreme relief (int64 slopes)
    (93, (560, 800), (1300, 1250), 2500),    # quadrant mode
    (94, (1100, 1600), (3300, 3200), 2700),  # global-bitmap mode
])
def test_viewshed_ray_per_wave(S, orc, seed, roi, shape, relief):
    # one wavefront per ray (64 samples at a time, the horizon as a prefix
    # maximum across lanes): the same bits as the oracle, edge windows included
    _say("viewshed ray per wave", seed, roi, shape)
    nr, nc = shape
    if relief is None:
        z = np.random.default_rng(seed).integers(-32768, 32767, size=shape).astype(np.int16)
        height = (0, 32767)
    else:
        z = _terrain(nr, 2.4, relief, seed, ncols=nc)
        height = (5, 100)
    obs = _quadrant_observers(nr, nc, 24, seed, roi, height)
    sc = S.Schedule(16, 1, 0, 1)
    got, want = _viewshed_case(S, orc, z, obs, roi[1], sched=sc)
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, ("viewshed words differ", bad[:8])
    if roi[1] <= 1087:
        vis, cells = S.siting_viewshed_batch(torch.from_numpy(z).cuda(),
                                             S.observers_to_device(obs), None, roi[1],
                                             sched=sc, sink=S.SITING_SINK_COUNT)
        wv, wc = orc.viewshed_count(z, obs)
        assert (vis.cpu().numpy().astype(np.uint32) == wv).all()
        assert (cells.cpu().numpy().astype(np.uint32) == wc).all()


def test_viewshed_wide_arithmetic(S, orc):
    # extreme relief forces the int64 comparison path
    rng = np.random.default_rng(0)
    z = rng.integers(-32768, 32767, size=(260, 270)).astype(np.int16)
    from synth import uniform_observers
    obs = uniform_observers(260, 270, 60, 9, roi=(60, 120), height=(0, 32767))
    got, want = _viewshed_case(S, orc, z, obs, 120)
    assert (got == want).all()


def test_viewshed_count_sink(S, orc):
    from synth import uniform_observers
    z = _terrain(400, 2.4, 1200, 21)
    obs = uniform_observers(400, 400, 150, 21, roi=(5, 110), height=(0, 50))
    zd = torch.from_numpy(z).cuda()
    vis, cells = S.siting_viewshed_batch(zd, S.observers_to_device(obs), None, 110,
                                         sink=S.SITING_SINK_COUNT)
    wv, wc = orc.viewshed_count(z, obs)
    assert (vis.cpu().numpy().astype(np.uint32) == wv).all()
    assert (cells.cpu().numpy().astype(np.uint32) == wc).all()


def test_autotune_returns_a_candidate(S, orc):
    from synth import uniform_observers
    z = _terrain(600, 2.4, 1000, 2)
    obs = uniform_observers(600, 600, 400, 2, roi=(100, 100), height=(10, 10))
    zd = torch.from_numpy(z).cuda()
    off = S.siting_viewshed_layout(obs, 600, 600)
    off_d = torch.from_numpy(off).cuda()
    obs_d = S.observers_to_device(obs)
    bm = torch.empty(int(off[-1]), dtype=torch.int64, device="cuda")
    best, times = S.siting_autotune(zd, obs_d, off_d, 100, bm)
    assert best.as_tuple() in [c.as_tuple() for c in S.siting_autotune_candidates(100)]
    assert all(t > 0 for t in times)
    want, _ = orc.viewshed(z, obs)
    assert (_u64(bm)[:off[-1]] == want).all()


# --------------------------------------------------------------- SITE ------
@pytest.mark.parametrize("seed,n_obs,max_obs,frac,roi", [
    (1, 400, 60, 1.0, (20, 90)), (2, 300, 1000, 0.5, (20, 90)), (3, 50, 200, 1.0, (20, 90)),
    (4, 3000, 400, 1.0, (5, 40)),     # dense: hundreds of windows meet each winner
    (5, 1, 5, 1.0, (30, 30)),         # a single candidate
    (6, 700, 300, 1.0, (1, 250)),     # very uneven ROIs (bucket side from the largest)
])
def test_greedy_parity(S, orc, seed, n_obs, max_obs, frac, roi):
    _say("greedy", seed, n_obs, max_obs, frac, roi)
    from synth import uniform_observers
    z = _terrain(500, 2.4, 1500, seed)
    obs = uniform_observers(500, 500, n_obs, seed, roi=roi, height=(5, 30))
    bm_h, off = orc.viewshed(z, obs)
    tgt = 500 * 500 if frac >= 1 else int(math.ceil(frac * 500 * 500))
    wsel, wgain, wcum, _ = orc.greedy(bm_h, off, obs, 500, 500, max_obs, tgt, lazy=True)
    bm = torch.from_numpy(bm_h.view(np.int64)).cuda()
    sel, gains, nsel, cum = S.siting_greedy(bm, torch.from_numpy(off).cuda(),
                                            S.observers_to_device(obs), 500, 500, max_obs, tgt)
    m = int(nsel.item())
    assert m == len(wsel)
    assert (sel[:m].cpu().numpy() == wsel).all()
    assert (gains[:m].cpu().numpy() == wgain).all()
    assert (_u64(cum).reshape(-1) == wcum.reshape(-1)).all()


@pytest.mark.parametrize("seed,n_obs,roi", [
    (11, 120, (400, 600)),   # every window spans several batches of every wavefront
    (12, 300, (5, 600)),     # small and large windows interleave
])
def test_greedy_large_windows(S, orc, seed, n_obs, roi):
    # windows above 1024 words run on four wavefronts; same selection as the
    # oracle's greedy over the oracle's own viewsheds
    _say("greedy large windows", seed, n_obs, roi)
    from synth import uniform_observers
    nr, nc = 1300, 1210
    z = _terrain(nr, 2.4, 1500, seed, ncols=nc)
    obs = uniform_observers(nr, nc, n_obs, seed, roi=roi, height=(5, 60))
    bm_h, off = orc.viewshed(z, obs)
    wsel, wgain, wcum, _ = orc.greedy(bm_h, off, obs, nr, nc, 150, nr * nc, lazy=True)
    bm = torch.from_numpy(bm_h.view(np.int64)).cuda()
    sel, gains, nsel, cum = S.siting_greedy(bm, torch.from_numpy(off).cuda(),
                                            S.observers_to_device(obs), nr, nc, 150, nr * nc)
    m = int(nsel.item())
    assert m == len(wsel)
    assert (sel[:m].cpu().numpy() == wsel).all()
    assert (gains[:m].cpu().numpy() == wgain).all()
    assert (_u64(cum).reshape(-1) == wcum.reshape(-1)).all()


@pytest.mark.parametrize("seed,nr,nc,n_obs,roi,max_obs", [
    (61, 500, 500, 600, (20, 90), 150),    # one-wavefront rounds
    (62, 900, 870, 300, (100, 400), 80),   # windows above 1024 words: four wavefronts
    (63, 400, 400, 2000, (5, 30), 400),    # many small windows; picks stop when none is seen
])
def test_greedy_intervisible_parity(S, orc, seed, nr, nc, n_obs, roi, max_obs):
    # intervisibility: after the first pick only candidates whose post lies in
    # the cumulative viewshed compete; selection, gains and cumulative
    # viewshed equal the oracle's on its own bitmaps
    _say("greedy intervisible", seed, nr, nc, n_obs, roi, max_obs)
    from synth import uniform_observers
    z = _terrain(nr, 2.4, 1500, seed, ncols=nc)
    obs = uniform_observers(nr, nc, n_obs, seed, roi=roi, height=(5, 40))
    bm_h, off = orc.viewshed(z, obs)
    wsel, wgain, wcum, _ = orc.greedy(bm_h, off, obs, nr, nc, max_obs, nr * nc, lazy=True,
                                      intervisible=True)
    bm = torch.from_numpy(bm_h.view(np.int64)).cuda()
    sel, gains, nsel, cum = S.siting_greedy(bm, torch.from_numpy(off).cuda(),
                                            S.observers_to_device(obs), nr, nc, max_obs, nr * nc,
                                            intervisible=True)
    m = int(nsel.item())
    _say("picks", m, "of", max_obs)
    assert m == len(wsel)
    assert (sel[:m].cpu().numpy() == wsel).all()
    assert (gains[:m].cpu().numpy() == wgain).all()
    assert (_u64(cum).reshape(-1) == wcum.reshape(-1)).all()


def test_greedy_intervisible_chain_on_flat_terrain(S, orc):
    # flat terrain, every viewshed its disk: A first, then B (in A's disk),
    # then C (only in B's); D far away never becomes eligible
    z = np.zeros((100, 100), np.int16)
    obs = orc.observers([50, 65, 74, 20], [50, 50, 50, 20], [20, 10, 10, 15], 5, 5)
    bm_h, off = orc.viewshed(z, obs)
    bm = torch.from_numpy(bm_h.view(np.int64)).cuda()
    sel, gains, nsel, _ = S.siting_greedy(bm, torch.from_numpy(off).cuda(),
                                          S.observers_to_device(obs), 100, 100, 10, 10**9,
                                          intervisible=True)
    assert int(nsel.item()) == 3 and sel[:3].cpu().tolist() == [0, 1, 2]


@pytest.mark.parametrize("seed,nr,nc,n_obs,roi,max_obs,batch", [
    (81, 1300, 1210, 150, (400, 600), 60, 1),     # one re-evaluation per round
    (81, 1300, 1210, 150, (400, 600), 60, 7),
    (82, 900, 870, 700, (5, 300), 250, 64),       # small and large windows
    (83, 500, 500, 2500, (20, 90), 400, 1024),    # more blocks than one batch holds
])
def test_greedy_parallel_parity(S, orc, seed, nr, nc, n_obs, roi, max_obs, batch):
    # rounds spread over the GPU: the same selection, gains and cumulative
    # viewshed as the oracle's greedy on its own bitmaps, whatever the batch
    _say("greedy parallel", seed, nr, nc, n_obs, roi, max_obs, batch)
    from synth import uniform_observers
    z = _terrain(nr, 2.4, 1500, seed, ncols=nc)
    obs = uniform_observers(nr, nc, n_obs, seed, roi=roi, height=(5, 60))
    bm_h, off = orc.viewshed(z, obs)
    wsel, wgain, wcum, _ = orc.greedy(bm_h, off, obs, nr, nc, max_obs, nr * nc, lazy=True)
    bm = torch.from_numpy(bm_h.view(np.int64)).cuda()
    sel, gains, nsel, cum = S.siting_greedy(bm, torch.from_numpy(off).cuda(),
                                            S.observers_to_device(obs), nr, nc, max_obs, nr * nc,
                                            parallel=batch)
    m = int(nsel.item())
    assert m == len(wsel)
    assert (sel[:m].cpu().numpy() == wsel).all()
    assert (gains[:m].cpu().numpy() == wgain).all()
    assert (_u64(cum).reshape(-1) == wcum.reshape(-1)).all()


def test_greedy_ties_on_flat_terrain(S, orc):
    # flat terrain: equal disks everywhere.  Observers on a lattice of spacing
    # 2R+1 never overlap, so every round is a tie among all unselected ones
    # and the selection is their indices in increasing order; a second group
    # overlaps the first and duplicates some of its posts (ties at lower
    # gains, and zero gains once a duplicate's twin is in).
    n, R = 300, 12
    z = np.full((n, n), 250, np.int16)
    rng = np.random.default_rng(3)
    pts = [(x, y) for y in range(R, n - R, 2 * R + 1) for x in range(R, n - R, 2 * R + 1)]
    rng.shuffle(pts)
    lattice = orc.observers([p[0] for p in pts], [p[1] for p in pts], R, 10, 10)
    bm_h, off = orc.viewshed(z, lattice)
    ones = np.bitwise_count(bm_h).astype(np.int64)
    sizes = np.add.reduceat(ones, off[:-1])
    assert (sizes == sizes[0]).all()          # every gain ties at first
    sel, gains, _ = _greedy_both(S, orc, z, lattice, len(lattice) + 5, n * n)
    assert (sel == np.arange(len(lattice))).all() and (gains == sizes[0]).all()
    dup = lattice[rng.permutation(len(lattice))[:20]]
    shifted = lattice[:30].copy()
    shifted["x"] += 6
    mixed = np.concatenate([dup, lattice, shifted, dup])
    sel, gains, _ = _greedy_both(S, orc, z, mixed, 200, n * n)
    assert (np.diff(gains) <= 0).all() and len(sel) < len(mixed)


def _greedy_both(S, orc, z, obs, max_obs, tgt):
    nr, nc = z.shape
    bm_h, off = orc.viewshed(z, obs)
    wsel, wgain, wcum, _ = orc.greedy(bm_h, off, obs, nr, nc, max_obs, tgt, lazy=True)
    psel, pgain, _ = orc.greedy(bm_h, off, obs, nr, nc, max_obs, tgt)
    assert (psel == wsel).all() and (pgain == wgain).all()
    zd = torch.from_numpy(z).cuda()
    obs_d = S.observers_to_device(obs)
    off_d = torch.from_numpy(off).cuda()
    bm = S.siting_viewshed_batch(zd, obs_d, off_d, int(obs["roi"].max()))
    assert (_u64(bm)[:off[-1]] == bm_h).all()
    sel, gains, nsel, cum = S.siting_greedy(bm, off_d, obs_d, nr, nc, max_obs, tgt)
    m = int(nsel.item())
    assert m == len(wsel)
    assert (sel[:m].cpu().numpy() == wsel).all() and (gains[:m].cpu().numpy() == wgain).all()
    assert (_u64(cum).reshape(-1) == wcum.reshape(-1)).all()
    return wsel, wgain, wcum


def test_visibility_index_labels(S, orc):
    # the exact visibility index (visible - 1) / (cells - 1) from the count
    # sink, clipped windows included, bit for bit against the oracle's
    # float32 quotient of its own counts
    from synth import uniform_observers
    z = _terrain(350, 2.4, 1500, 23)
    obs = uniform_observers(350, 350, 400, 23, roi=(1, 120), height=(0, 40))
    vis, cells = S.siting_viewshed_batch(torch.from_numpy(z).cuda(), S.observers_to_device(obs),
                                         None, 120, sink=S.SITING_SINK_COUNT)
    vi = S.siting_visibility_index(vis[:len(obs)], cells[:len(obs)]).cpu().numpy()
    want = orc.visibility_index(z, obs)
    assert vi.dtype == np.float32 and (vi.view(np.uint32) == want.view(np.uint32)).all()
    assert (vi >= 0).all() and (vi <= 1).all()


# ------------------------------------------------------------- PIPELINE ----
def test_pipeline_plain_1000_end_to_end(S, orc):
    from paper_2006_16783_amd import pipeline as P
    cfg = P.CONFIGS["plain_1000"]
    z = _terrain(cfg.n, cfg.beta, cfg.zmax, cfg.seed)
    zd = torch.from_numpy(z).cuda()
    res = P.run(zd, cfg)
    cnt = orc.vix(z, cfg.roi, cfg.h_t, cfg.h_r, cfg.K, cfg.vix_seed)
    cand = orc.findmax(cnt, z, cfg.grid, cfg.grid, cfg.k)
    cand = cand[cand >= 0]
    assert (res.candidates == cand).all()
    obs = orc.observers(cand % cfg.n, cand // cfg.n, cfg.roi, cfg.h_t, cfg.h_r)
    bm, off = orc.viewshed(z, obs)
    sel, gains, cum = orc.greedy(bm, off, obs, cfg.n, cfg.n, cfg.max_obs,
                                 P.target_cells(cfg.target_frac, cfg.n, cfg.n))
    assert (res.selected == sel).all() and (res.gains == gains).all()
    # coverage is non-decreasing and equals the union's popcount
    assert (np.diff(res.gains) <= 0).all()
    assert res.coverage_cells == sum(bin(int(v)).count("1") for v in cum.ravel())


def _oracle_site_positions(orc, z, cfg):
    """The oracle's chain VIX -> FINDMAX -> VIEWSHED -> greedy SITE on terrain
    z (host int16): the chosen posts' (x, y)."""
    from paper_2006_16783_amd import pipeline as P
    nr, nc = z.shape
    cnt = orc.vix(z, cfg.roi, cfg.h_t, cfg.h_r, cfg.K, cfg.vix_seed)
    cand = orc.findmax(cnt, z, cfg.grid, cfg.grid, cfg.k)
    cand = cand[cand >= 0]
    obs = orc.observers(cand % nc, cand // nc, cfg.roi, cfg.h_t, cfg.h_r)
    bm, off = orc.viewshed(z, obs)
    sel, _, _, _ = orc.greedy(bm, off, obs, nr, nc, cfg.max_obs,
                              P.target_cells(cfg.target_frac, nr, nc), lazy=True)
    return obs["x"][sel].astype(np.int64), obs["y"][sel].astype(np.int64)


def _oracle_union(orc, z, xs, ys, cfg):
    """Cells of terrain z seen by observers at (xs, ys): the OR of their
    oracle viewsheds, counted."""
    nr, nc = z.shape
    obs = orc.observers(xs, ys, cfg.roi, cfg.h_t, cfg.h_r)
    bm, off = orc.viewshed(z, obs)
    C = np.zeros((nr, (nc + 63) // 64), np.uint64)
    for i, o in enumerate(obs):
        R, x, y = int(o["roi"]), int(o["x"]), int(o["y"])
        ylo, yhi = max(0, y - R), min(nr - 1, y + R)
        w0, w1 = max(0, x - R) >> 6, min(nc - 1, x + R) >> 6
        C[ylo:yhi + 1, w0:w1 + 1] |= bm[off[i]:off[i + 1]].reshape(yhi - ylo + 1, w1 - w0 + 1)
    return int(np.bitwise_count(C).sum())


@pytest.mark.parametrize("q,f", [(1, 1), (10, 1), (50, 1), (1, 2), (1, 4)])
def test_lowered_accuracy_against_oracle(S, orc, q, f):
    # the 1000^2 workload (ROI 100, h 10/10, K 10, 10x10 blocks x 10, SITE to
    # 100) sited on a degraded terrain -- elevations quantised to q m, or
    # every f-th post with the ROI divided by f -- and scored on the full
    # terrain: the chosen posts and the union area of their viewsheds there
    # equal the oracle's chain on the same degraded array
    import dataclasses
    from paper_2006_16783_amd import accuracy as A
    from paper_2006_16783_amd import pipeline as P
    _say("accuracy", q, f)
    cfg = P.CONFIGS["plain_1000"]
    z = _terrain(cfg.n, cfg.beta, cfg.zmax, cfg.seed)
    zd = torch.from_numpy(z).cuda()
    xs, ys, _, res = A.site_degraded(zd, cfg, q, f)
    area = A.union_area(zd, xs, ys, cfg)
    # the oracle on the same degraded terrain (host arithmetic on the array)
    zq = (z // q * q).astype(np.int16) if q > 1 else z
    c = cfg
    if f > 1:
        zq = np.ascontiguousarray(zq[::f, ::f])
        c = dataclasses.replace(cfg, n=zq.shape[0], roi=max(1, cfg.roi // f),
                                grid=min(cfg.grid, zq.shape[0]))
    oxs, oys = _oracle_site_positions(orc, zq, c)
    assert len(oxs) == len(xs) > 0
    assert (oxs * f == xs).all() and (oys * f == ys).all()
    want = _oracle_union(orc, z, xs, ys, cfg)
    assert area == want
    if (q, f) == (1, 1):
        # the exact run's own choice scores exactly its coverage
        assert area == res.coverage_cells
    _say("accuracy", q, f, "observers", len(xs), "area", area)