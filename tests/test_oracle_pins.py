"""Pins of the CPU oracle against things other than itself: published
generator known answers, the paper's printed block counts, closed forms, invariants and a
pure-Python brute force with exact rational arithmetic (tests/brute.py)."""
import math
import os

import numpy as np
import pytest

import brute
from synth import fbm, uniform_observers

HERE = os.path.dirname(os.path.abspath(__file__))


def _rand_terrain(rng, nr, nc, lo=0, hi=40):
    return rng.integers(lo, hi + 1, size=(nr, nc)).astype(np.int16)


# ---------------------------------------------------------------- RNG ------
def _kat_rows():
    rows = []
    for line in open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")):
        if line.strip() and not line.startswith("#"):
            w = [int(v, 16) for v in line.split()]
            assert len(w) == 10
            rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


def test_philox4x32_known_answers(orc):
    rows = _kat_rows()
    assert len(rows) == 3
    for ctr, key, want in rows:
        got = orc.philox4x32_10(np.array(ctr, np.uint32), np.array(key, np.uint32))
        assert [int(v) for v in got] == want, (ctr, key)


# ---------------------------------------------------------------- LOS ------
def test_los_brute_force_all_pairs(orc):
    rng = np.random.default_rng(11)
    for trial in range(6):
        nr, nc = int(rng.integers(5, 11)), int(rng.integers(5, 11))
        z = _rand_terrain(rng, nr, nc, 0, 30)
        zl = z.tolist()
        h_t, h_r = int(rng.integers(0, 6)), int(rng.integers(0, 6))
        for ty in range(nr):
            for tx in range(nc):
                for py in range(nr):
                    for px in range(nc):
                        a = orc.los(z, (tx, ty), (px, py), h_t, h_r)
                        b = brute.los(zl, (tx, ty), (px, py), h_t, h_r)
                        assert a == b, (trial, tx, ty, px, py)


def test_los_flat_and_symmetry(orc):
    z = np.full((9, 12), 7, np.int16)
    for p in [(0, 0), (11, 8), (5, 0), (11, 3)]:
        assert orc.los(z, (4, 4), p, 0, 0)
    rng = np.random.default_rng(3)
    z = _rand_terrain(rng, 12, 12, 0, 50)
    for _ in range(300):
        t = tuple(int(v) for v in rng.integers(0, 12, 2))
        p = tuple(int(v) for v in rng.integers(0, 12, 2))
        h = int(rng.integers(0, 10))
        # the same segment and grid-line crossings in both directions
        assert orc.los(z, t, p, h, h) == orc.los(z, p, t, h, h)


def test_los_single_wall_closed_form(orc):
    # flat z=0, a wall of height W in column tx+a; receiver in row ty at dx>a:
    # visible iff the segment at the wall, h_t + (h_r-h_t)*a/dx, is >= W.
    nr, nc, tx, ty = 5, 40, 2, 2
    for W in (3, 10, 25):
        for a in (1, 3, 7):
            z = np.zeros((nr, nc), np.int16)
            z[:, tx + a] = W
            for h_t, h_r in [(5, 1), (20, 2), (30, 30), (1, 40)]:
                for dx in range(a + 1, nc - tx):
                    want = h_t * dx + (h_r - h_t) * a >= W * dx
                    assert orc.los(z, (tx, ty), (tx + dx, ty), h_t, h_r) == want


def test_los_monotone_in_heights(orc):
    rng = np.random.default_rng(5)
    z = _rand_terrain(rng, 16, 16, 0, 60)
    for _ in range(400):
        t = tuple(int(v) for v in rng.integers(0, 16, 2))
        p = tuple(int(v) for v in rng.integers(0, 16, 2))
        h1, h2 = sorted(int(v) for v in rng.integers(0, 30, 2))
        assert orc.los(z, t, p, h1, 5) <= orc.los(z, t, p, h2, 5)
        assert orc.los(z, t, p, 5, h1) <= orc.los(z, t, p, 5, h2)


# ---------------------------------------------------------------- VIX ------
def test_vix_targets_valid_and_counted(orc):
    rng = np.random.default_rng(8)
    z = _rand_terrain(rng, 20, 17, 0, 40)
    R, K, seed = 6, 12, 99
    cnt = orc.vix(z, R, 3, 2, K, seed)
    zl = z.tolist()
    for y in range(20):
        for x in range(17):
            tx, ty = orc.vix_targets(20, 17, x, y, R, K, seed)
            c = 0
            for px, py in zip(tx.tolist(), ty.tolist()):
                assert px >= 0
                assert (px, py) != (x, y)
                assert (px - x) ** 2 + (py - y) ** 2 <= R * R
                assert 0 <= px < 17 and 0 <= py < 20
                c += brute.los(zl, (x, y), (px, py), 3, 2)
            assert c == cnt[y, x]


def test_vix_draw_stream_layout(orc):
    # post t's words: word a = word (a mod 4) of the Philox4x32-10 block
    # {t lo, a//4, t hi, 0} keyed {seed lo, seed hi} (the block function is
    # pinned by its known answers above); each word proposes one receiver, its
    # two 16-bit halves scaled to the clipped box by Lemire's multiply-shift
    # with rejection; draws take the accepted proposals in order.  A seed above
    # 2^32 and a post index above 2^32 check the word split of both.
    cases = [((50, 60), 7, 1234, [(0, 0), (30, 20), (59, 49), (3, 45)]),
             ((3, 2**31), 1, (7 << 32) | 5, [(2**31 - 1, 2), (2**31 - 3, 1)]),
             ((900, 900), 300, 77, [(450, 450), (0, 899)])]
    for (nr, nc), R, seed, posts in cases:
        key = np.array([seed & 0xffffffff, seed >> 32], np.uint32)
        for (x, y) in posts:
            tx, ty = orc.vix_targets(nr, nc, x, y, R, 9, seed)
            t = y * nc + x
            bx0, bx1 = max(0, x - R), min(nc - 1, x + R)
            by0, by1 = max(0, y - R), min(nr - 1, y + R)
            wx, wy = bx1 - bx0 + 1, by1 - by0 + 1
            words = []
            for b in range(60):
                ctr = np.array([t & 0xffffffff, b, t >> 32, 0], np.uint32)
                words += [int(w) for w in orc.philox4x32_10(ctr, key)]
            a = 0
            for j in range(9):
                # at most 64 proposals per draw; a draw with none accepted
                # fails (-1) and the next draw starts at the following word
                px = py = -1
                for _ in range(64):
                    u = words[a]
                    a += 1
                    mx, my = (u & 0xffff) * wx, (u >> 16) * wy
                    if (mx & 0xffff) < 65536 % wx or (my & 0xffff) < 65536 % wy:
                        continue
                    qx, qy = bx0 + (mx >> 16), by0 + (my >> 16)
                    if (qx, qy) != (x, y) and (qx - x) ** 2 + (qy - y) ** 2 <= R * R:
                        px, py = qx, qy
                        break
                assert (tx[j], ty[j]) == (px, py), (x, y, j)


def test_vix_rowlist_equals_whole_terrain_rows(orc):
    z = fbm(90, 2.4, 600, 4)
    full = orc.vix(z, 12, 5, 3, 7, 31)
    rows = [89, 0, 44, 45, 3]
    assert (orc.vix_rows(z, 12, 5, 3, 7, 31, rows) == full[rows]).all()


def test_lemire_scaling_is_exactly_uniform():
    # the box scaling of one coordinate: every 16-bit field value either
    # rejected or mapped, each of the w outputs hit by exactly floor(2^16/w)
    # values (the property that makes the draw exactly uniform)
    for w in (1, 3, 201, 255, 256, 257, 1000, 8189):
        t = 65536 % w
        hits = np.zeros(w, np.int64)
        for f in range(65536):
            m = f * w
            if (m & 0xffff) >= t:
                hits[m >> 16] += 1
        assert (hits == 65536 // w).all(), w


def test_vix_flat_is_full_and_monotone(orc):
    z = np.full((30, 30), 100, np.int16)
    assert (orc.vix(z, 8, 0, 0, 10, 1) == 10).all()
    z = fbm(48, 2.4, 300, 2)
    a = orc.vix(z, 10, 2, 2, 16, 5).astype(int)
    b = orc.vix(z, 10, 20, 2, 16, 5).astype(int)
    c = orc.vix(z, 10, 20, 30, 16, 5).astype(int)
    assert (a <= b).all() and (b <= c).all()


def test_vix_targets_uniform_chi2(orc):
    # draws of one interior post over many seeds: chi-square over disk cells
    R, nr, nc, x, y = 4, 20, 20, 10, 10
    cells = sorted((dx, dy) for dx in range(-R, R + 1) for dy in range(-R, R + 1)
                   if (dx, dy) != (0, 0) and dx * dx + dy * dy <= R * R)
    idx = {c: i for i, c in enumerate(cells)}
    counts = np.zeros(len(cells))
    for seed in range(200):
        tx, ty = orc.vix_targets(nr, nc, x, y, R, 40, seed)
        for px, py in zip(tx.tolist(), ty.tolist()):
            counts[idx[(px - x, py - y)]] += 1
    e = counts.sum() / len(cells)
    chi2 = float(((counts - e) ** 2 / e).sum())
    dof = len(cells) - 1
    # mean dof, sd sqrt(2 dof): 5 sigma bound
    assert chi2 < dof + 5 * math.sqrt(2 * dof)


def test_vix_clipped_corner_draws(orc):
    tx, ty = orc.vix_targets(3, 3, 0, 0, 50, 100, 7)
    for px, py in zip(tx.tolist(), ty.tolist()):
        assert 0 <= px < 3 and 0 <= py < 3 and (px, py) != (0, 0)
    seen = set(zip(tx.tolist(), ty.tolist()))
    assert seen == {(a, b) for a in range(3) for b in range(3)} - {(0, 0)}


# ------------------------------------------------------------ FINDMAX ------
def test_block_grid_matches_paper_tables(orc):
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "paper_blocks.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 5
    for n, roi, g, k, m in [[int(v) for v in r] for r in rows]:
        assert orc.block_grid(n, roi) == g
        assert g * g * k == m


def _findmax_numpy(key, z, gr, gc, k):
    nr, nc = z.shape
    out = []
    for bi in range(gr):
        for bj in range(gc):
            r0, r1 = bi * nr // gr, (bi + 1) * nr // gr
            c0, c1 = bj * nc // gc, (bj + 1) * nc // gc
            yy, xx = np.mgrid[r0:r1, c0:c1]
            idx = (yy * nc + xx).ravel()
            kk = key[r0:r1, c0:c1].ravel().astype(np.int64)
            zz = z[r0:r1, c0:c1].ravel().astype(np.int64)
            order = np.lexsort((idx, -zz, -kk))
            top = idx[order][:k].tolist()
            out += top + [-1] * (k - len(top))
    return np.array(out, np.int64)


@pytest.mark.parametrize("shape,gr,gc,k", [((37, 41), 3, 4, 5), ((20, 20), 5, 5, 20),
                                           ((64, 30), 7, 2, 3), ((9, 9), 9, 9, 2)])
def test_findmax_lexsort(orc, shape, gr, gc, k):
    rng = np.random.default_rng(shape[0] * 7 + k)
    key = rng.integers(0, 4, size=shape).astype(np.uint8)   # many ties
    z = rng.integers(0, 5, size=shape).astype(np.int16)
    assert (orc.findmax(key, z, gr, gc, k) == _findmax_numpy(key, z, gr, gc, k)).all()


def test_findmax_f32_strided(orc):
    rng = np.random.default_rng(4)
    z = rng.integers(0, 9, size=(23, 29)).astype(np.int16)       # many elevation ties
    s = 3
    kr, kc = -(-23 // s), -(-29 // s)
    sc = rng.integers(0, 5, size=(kr, kc)).astype(np.float32)
    sc[1, 2] = np.nan
    got = orc.findmax(sc, z, 2, 3, 4, stride=s)
    for b in range(6):
        bi, bj = divmod(b, 3)
        r0, r1 = bi * 23 // 2, (bi + 1) * 23 // 2
        c0, c1 = bj * 29 // 3, (bj + 1) * 29 // 3
        items = []
        for y in range(r0, r1):
            for x in range(c0, c1):
                if y % s == 0 and x % s == 0:
                    v = float(sc[y // s, x // s])
                    items.append((-(v if v == v else -np.inf), y * 29 + x))
        items.sort()
        # each winning cell stands for its highest post (elevation desc, index asc)
        want = []
        for _, i in items[:4]:
            y0, x0 = divmod(i, 29)
            cell = [(-int(z[y, x]), y * 29 + x) for y in range(y0, min(y0 + s, 23))
                    for x in range(x0, min(x0 + s, 29))]
            want.append(min(cell)[1])
        want += [-1] * max(0, 4 - len(items))
        assert got[b * 4:(b + 1) * 4].tolist() == want


# ----------------------------------------------------------- VIEWSHED ------
def _obs(orc, x, y, R, ht, hr):
    return orc.observers([x], [y], [R], [ht], [hr])


def test_viewshed_brute_force_tiny(orc):
    rng = np.random.default_rng(21)
    for trial in range(40):
        nr, nc = int(rng.integers(4, 26)), int(rng.integers(4, 26))
        z = _rand_terrain(rng, nr, nc, 0, int(rng.integers(1, 60)))
        x, y = int(rng.integers(0, nc)), int(rng.integers(0, nr))
        R = int(rng.integers(1, 14))
        ht, hr = int(rng.integers(0, 12)), int(rng.integers(0, 12))
        ob = _obs(orc, x, y, R, ht, hr)
        got = brute.bitmap_to_set(orc.viewshed_one(z, ob), nr, nc, (x, y, R))
        want = brute.viewshed(z.tolist(), (x, y, R, ht, hr))
        assert got == want, trial


def test_viewshed_flat_is_disk(orc):
    for (nr, nc, x, y, R) in [(40, 40, 20, 20, 13), (30, 70, 0, 5, 9), (25, 25, 24, 24, 30),
                              (130, 150, 64, 70, 60)]:
        z = np.full((nr, nc), 55, np.int16)
        ob = _obs(orc, x, y, R, 0, 0)
        got = brute.bitmap_to_set(orc.viewshed_one(z, ob), nr, nc, (x, y, R))
        assert got == brute.disk(nr, nc, x, y, R)


def test_viewshed_every_disk_cell_visited(orc):
    # with an enormous receiver height every visited cell is visible, so the
    # bitmap is exactly the set of cells some ray reaches: the whole disk.
    z = fbm(160, 2.2, 900, 3)
    for (x, y, R) in [(80, 80, 70), (0, 80, 45), (159, 3, 100), (40, 120, 1), (90, 60, 2)]:
        ob = _obs(orc, x, y, R, 0, 30000)
        got = brute.bitmap_to_set(orc.viewshed_one(z, ob), 160, 160, (x, y, R))
        assert got == brute.disk(160, 160, x, y, R)


def test_viewshed_single_wall(orc):
    nr, nc, tx, ty, R = 61, 61, 30, 30, 28
    for W, a, ht, hr in [(40, 4, 10, 5), (12, 9, 10, 10), (100, 2, 50, 1)]:
        z = np.zeros((nr, nc), np.int16)
        z[:, tx + a] = W
        ob = _obs(orc, tx, ty, R, ht, hr)
        vis = brute.bitmap_to_set(orc.viewshed_one(z, ob), nr, nc, (tx, ty, R))
        for dy in range(-R, R + 1):
            for dx in range(1, R + 1):
                if dx * dx + dy * dy > R * R or abs(dy) >= dx:
                    continue
                cell = (tx + dx, ty + dy)
                if dx < a:
                    assert cell in vis
                elif dx > a:
                    assert (cell in vis) == ((hr - ht) * a >= (W - ht) * dx), (W, a, cell)


def test_viewshed_one_side_clipped_equals_los(orc):
    # observer d columns from the right edge: cells (d, m) with |m| < d are
    # marked only by their own ray, at a step where the ray passes exactly
    # through them, so the bitmap equals per-cell line of sight there.
    z = fbm(120, 2.4, 600, 9)
    for d, R, ht, hr in [(12, 30, 5, 2), (25, 40, 1, 1), (7, 7, 10, 0)]:
        x, y = 119 - d, 60
        ob = _obs(orc, x, y, R, ht, hr)
        vis = brute.bitmap_to_set(orc.viewshed_one(z, ob), 120, 120, (x, y, R))
        for m in range(-d + 1, d):
            if d * d + m * m > R * R:
                continue
            cell = (x + d, y + m)
            assert (cell in vis) == orc.los(z, (x, y), cell, ht, hr)


def test_viewshed_ray_steps_through_cells_equal_los(orc):
    # brute per-ray dump: at a step with no fractional offset the ray's
    # verdict is per-cell line of sight to that cell (the horizon is the
    # maximum slope of exactly the samples that LOS tests).
    z = fbm(64, 2.2, 400, 4)
    zl = z.tolist()
    x, y, R, ht, hr = 30, 33, 25, 6, 3
    x0, x1, y0, y1 = brute.window(64, 64, x, y, R)
    for by in range(y0, y1 + 1):
        for bx in range(x0, x1 + 1):
            if not (bx in (x0, x1) or by in (y0, y1)):
                continue
            dump = []
            brute.ray(zl, 64, 64, (x, y, R, ht, hr), bx, by, dump)
            for k, frac, cell, vis in dump:
                if frac == 0:
                    assert vis == brute.los(zl, (x, y), cell, ht, hr)


def test_viewshed_monotone_ring_and_d4(orc):
    z = fbm(90, 2.4, 700, 12)
    x, y, R = 40, 47, 30
    sets = {}
    for ht, hr in [(2, 2), (10, 2), (10, 9)]:
        ob = _obs(orc, x, y, R, ht, hr)
        sets[(ht, hr)] = brute.bitmap_to_set(orc.viewshed_one(z, ob), 90, 90, (x, y, R))
    assert sets[(2, 2)] <= sets[(10, 2)] <= sets[(10, 9)]
    ring = {(x + a, y + b) for a in (-1, 0, 1) for b in (-1, 0, 1)}
    assert ring <= sets[(2, 2)]
    base = sets[(10, 2)]
    # the 8 symmetries of the square, applied to terrain and observer
    for tr in range(8):
        zt = z.T if tr & 4 else z
        px, py = (y, x) if tr & 4 else (x, y)
        if tr & 1:
            zt = zt[:, ::-1]; px = 89 - px
        if tr & 2:
            zt = zt[::-1, :]; py = 89 - py
        zt = np.ascontiguousarray(zt)
        ob = _obs(orc, px, py, R, 10, 2)
        got = brute.bitmap_to_set(orc.viewshed_one(zt, ob), 90, 90, (px, py, R))

        def fwd(c):
            cx, cy = (c[1], c[0]) if tr & 4 else c
            if tr & 1:
                cx = 89 - cx
            if tr & 2:
                cy = 89 - cy
            return (cx, cy)
        assert got == {fwd(c) for c in base}, tr


def test_viewshed_r3_brute_force_tiny(orc):
    # the exact per-cell viewshed: every disk cell by the rational LOS of
    # tests/brute.py, the observer's own cell visible
    rng = np.random.default_rng(31)
    for trial in range(40):
        nr, nc = int(rng.integers(4, 24)), int(rng.integers(4, 24))
        z = _rand_terrain(rng, nr, nc, 0, int(rng.integers(1, 60)))
        x, y = int(rng.integers(0, nc)), int(rng.integers(0, nr))
        R = int(rng.integers(1, 12))
        ht, hr = int(rng.integers(0, 12)), int(rng.integers(0, 12))
        ob = _obs(orc, x, y, R, ht, hr)
        bm, off = orc.viewshed_r3(z, ob)
        got = brute.bitmap_to_set(bm.reshape(-1, _nw(nc, x, R)), nr, nc, (x, y, R))
        zl = z.tolist()
        want = {c for c in brute.disk(nr, nc, x, y, R)
                if c == (x, y) or brute.los(zl, (x, y), c, ht, hr)}
        assert got == want, trial


def _nw(nc, x, R):
    return (min(nc - 1, x + R) >> 6) - (max(0, x - R) >> 6) + 1


def test_viewshed_r3_flat_is_disk_and_wall(orc):
    for (nr, nc, x, y, R, ht, hr) in [(40, 40, 20, 20, 13, 0, 0), (30, 70, 0, 5, 9, 7, 2),
                                      (25, 25, 24, 24, 30, 0, 9)]:
        z = np.full((nr, nc), 55, np.int16)
        bm, _ = orc.viewshed_r3(z, _obs(orc, x, y, R, ht, hr))
        got = brute.bitmap_to_set(bm.reshape(-1, _nw(nc, x, R)), nr, nc, (x, y, R))
        assert got == brute.disk(nr, nc, x, y, R)
    # a wall of height W one column a to the right: an x-major cell dx > a
    # away is visible iff (hr - ht) * a >= (W - ht) * dx
    nr, nc, tx, ty, R = 61, 61, 30, 30, 28
    for W, a, ht, hr in [(40, 4, 10, 5), (12, 9, 10, 10)]:
        z = np.zeros((nr, nc), np.int16)
        z[:, tx + a] = W
        bm, _ = orc.viewshed_r3(z, _obs(orc, tx, ty, R, ht, hr))
        vis = brute.bitmap_to_set(bm.reshape(-1, _nw(nc, tx, R)), nr, nc, (tx, ty, R))
        for dy in range(-R, R + 1):
            for dx in range(a + 1, R + 1):
                if dx * dx + dy * dy <= R * R and abs(dy) <= dx:
                    assert ((tx + dx, ty + dy) in vis) == ((hr - ht) * a >= (W - ht) * dx)


def test_viewshed_batch_layout_and_count(orc):
    z = fbm(100, 2.4, 500, 6)
    obs = uniform_observers(100, 100, 25, 3, roi=(3, 40), height=(0, 20))
    bm, off = orc.viewshed(z, obs)
    vis, cells = orc.viewshed_count(z, obs)
    for i, o in enumerate(obs):
        one = orc.viewshed_one(z, o)
        assert (bm[off[i]:off[i + 1]] == one.ravel()).all()
        assert vis[i] == sum(bin(int(v)).count("1") for v in one.ravel())
        assert cells[i] == len(brute.disk(100, 100, int(o["x"]), int(o["y"]), int(o["roi"])))


# --------------------------------------------------------------- SITE ------
def _sets_from(orc, z, obs):
    nr, nc = z.shape
    bm, off = orc.viewshed(z, obs)
    sets = []
    for i, o in enumerate(obs):
        w = bm[off[i]:off[i + 1]]
        R = int(o["roi"])
        x0 = max(0, int(o["x"]) - R)
        nw = ((min(nc - 1, int(o["x"]) + R)) >> 6) - (x0 >> 6) + 1
        sets.append(brute.bitmap_to_set(w.reshape(-1, nw), nr, nc,
                                        (int(o["x"]), int(o["y"]), R)))
    return bm, off, sets


def test_greedy_brute_lazy_and_invariants(orc):
    for seed in range(4):
        z = fbm(80, 2.4, 400, 30 + seed)
        obs = uniform_observers(80, 80, 30, seed, roi=(4, 25), height=(1, 15))
        bm, off, sets = _sets_from(orc, z, obs)
        target = int(math.ceil(0.9 * 80 * 80))
        sel, gains, cum = orc.greedy(bm, off, obs, 80, 80, 20, target)
        bsel, bgains, bcov = brute.greedy_sets(sets, 20, target)
        assert sel.tolist() == bsel and gains.tolist() == bgains
        lsel, lgains, lcum, evals = orc.greedy(bm, off, obs, 80, 80, 20, target, lazy=True)
        assert lsel.tolist() == sel.tolist() and lgains.tolist() == gains.tolist()
        assert (lcum == cum).all()
        # gains never grow (submodularity); sum of gains is the union's area
        assert all(gains[i] >= gains[i + 1] for i in range(len(gains) - 1))
        pop = sum(bin(int(v)).count("1") for v in cum.ravel())
        assert pop == int(gains.sum()) == len(bcov)


def test_greedy_stop_rules(orc):
    z = fbm(64, 2.4, 300, 1)
    obs = uniform_observers(64, 64, 12, 2, roi=(5, 30), height=(2, 10))
    bm, off, sets = _sets_from(orc, z, obs)
    sel, gains, _ = orc.greedy(bm, off, obs, 64, 64, 5, 10**9)
    assert len(sel) == 5
    sel, gains, _ = orc.greedy(bm, off, obs, 64, 64, 100, 10**9)
    # stops at zero gain: every candidate's cells are covered
    u = set().union(*sets)
    assert int(gains.sum()) == len(u) and len(sel) <= 12
    tgt = int(gains[0]) + 1
    sel2, gains2, _ = orc.greedy(bm, off, obs, 64, 64, 100, tgt)
    assert len(sel2) == 2


def test_greedy_intervisible_brute_and_lazy(orc):
    # intervisibility: after the first pick a candidate competes only if its
    # post is covered; the oracle (plain and lazy) against greedy over Python
    # sets with that rule, and every later pick lies in the union of the
    # viewsheds chosen before it
    for seed in range(5):
        z = fbm(90, 2.4, 500, 40 + seed)
        obs = uniform_observers(90, 90, 40, 10 + seed, roi=(4, 22), height=(1, 12))
        bm, off, sets = _sets_from(orc, z, obs)
        posts = [(int(o["x"]), int(o["y"])) for o in obs]
        target = int(math.ceil(0.95 * 90 * 90))
        sel, gains, cum = orc.greedy(bm, off, obs, 90, 90, 30, target, intervisible=True)
        bsel, bgains, bcov = brute.greedy_sets_intervisible(sets, posts, 30, target)
        assert sel.tolist() == bsel and gains.tolist() == bgains
        lsel, lgains, lcum, _ = orc.greedy(bm, off, obs, 90, 90, 30, target, lazy=True,
                                          intervisible=True)
        assert lsel.tolist() == bsel and lgains.tolist() == bgains and (lcum == cum).all()
        seen = set()
        for t, i in enumerate(bsel):
            assert t == 0 or posts[i] in seen
            seen |= sets[i]
        pop = sum(bin(int(v)).count("1") for v in cum.ravel())
        assert pop == int(gains.sum()) == len(bcov)


def test_greedy_intervisible_chain_on_flat_terrain(orc):
    # flat terrain: every viewshed is its whole disk.  A (R 20) is picked
    # first; B lies in A's disk, C only in B's, D (R 15) far from all: with
    # intervisibility the picks are A, B, C and D never becomes eligible;
    # without it D's larger disk is picked second
    z = np.zeros((100, 100), np.int16)
    obs = orc.observers([50, 65, 74, 20], [50, 50, 50, 20], [20, 10, 10, 15], 5, 5)
    bm, off = orc.viewshed(z, obs)
    sel, gains, _ = orc.greedy(bm, off, obs, 100, 100, 10, 10**9, intervisible=True)
    assert sel.tolist() == [0, 1, 2]
    disk = lambda R: sum(1 for dx in range(-R, R + 1) for dy in range(-R, R + 1)
                         if dx * dx + dy * dy <= R * R)
    assert gains[0] == disk(20)
    free, fgains, _ = orc.greedy(bm, off, obs, 100, 100, 10, 10**9)
    assert free.tolist()[:2] == [0, 3] and fgains[1] == disk(15)


def test_greedy_approximation_bound(orc):
    # greedy >= (1 - 1/e) of the exhaustive optimum (Nemhauser-Wolsey-Fisher)
    for seed in range(3):
        z = fbm(48, 2.4, 300, 50 + seed)
        obs = uniform_observers(48, 48, 10, 70 + seed, roi=(4, 16), height=(1, 6))
        bm, off, sets = _sets_from(orc, z, obs)
        for m in (2, 3):
            sel, gains, _ = orc.greedy(bm, off, obs, 48, 48, m, 10**9)
            opt = brute.best_cover(sets, m)
            assert int(gains.sum()) >= (1 - 1 / math.e) * opt
