"""Pure-Python brute force for tiny terrains, used to pin the C oracle.

Written independently of the oracle: heights and slopes are exact Fractions
(not cross-multiplied integers), rays are enumerated per boundary cell with
Python sets, and greedy works on Python sets of (x, y) cells.
"""
from __future__ import annotations

from fractions import Fraction
from itertools import combinations


def _sign(v):
    return -1 if v < 0 else 1


def los(z, t, p, h_t, h_r) -> bool:
    """Segment from the eye above t to the receiver top above p, tested at
    every crossing of a major-axis grid line against the terrain linearly
    interpolated between the two posts that bracket the crossing."""
    (tx, ty), (px, py) = t, p
    dx, dy = px - tx, py - ty
    E = Fraction(int(z[ty][tx]) + h_t)
    Zt = Fraction(int(z[py][px]) + h_r)
    xmaj = abs(dx) >= abs(dy)
    n = abs(dx) if xmaj else abs(dy)
    if n <= 1:
        return True
    for k in range(1, n):
        f = Fraction(k, n)
        if xmaj:
            x = tx + _sign(dx) * k
            yc = Fraction(ty) + dy * f          # exact crossing
            ylo = (yc.numerator // yc.denominator)
            w = yc - ylo
            zt = z[ylo][x] * (1 - w) + (z[ylo + 1][x] * w if w else 0)
        else:
            y = ty + _sign(dy) * k
            xc = Fraction(tx) + dx * f
            xlo = (xc.numerator // xc.denominator)
            w = xc - xlo
            zt = z[y][xlo] * (1 - w) + (z[y][xlo + 1] * w if w else 0)
        seg = E + (Zt - E) * f
        if zt > seg:
            return False
    return True


def window(nrows, ncols, x, y, R):
    return max(0, x - R), min(ncols - 1, x + R), max(0, y - R), min(nrows - 1, y + R)


def ray(z, nrows, ncols, ob, bx, by, dump=None):
    """One sweep ray; returns the set of cells it marks visible.  When dump is
    a list, (k, r, cell, visible) is appended per step."""
    x, y, R, h_t, h_r = ob
    dx, dy = bx - x, by - y
    xmaj = abs(dx) >= abs(dy)
    n = abs(dx) if xmaj else abs(dy)
    mn = abs(dy) if xmaj else abs(dx)
    sx, sy = _sign(dx), _sign(dy)
    E = Fraction(int(z[y][x]) + h_t)
    horizon = None                     # max slope of terrain samples so far
    out = set()
    for k in range(1, n + 1):
        pos = Fraction(k * mn, n)      # exact minor offset of the crossing
        q = pos.numerator // pos.denominator
        frac = pos - q
        m = q + (1 if frac >= Fraction(1, 2) else 0)
        if k * k + m * m > R * R:
            break
        if xmaj:
            px, py0, py1 = x + sx * k, y + sy * q, y + sy * (q + 1)
            terr = z[py0][px] * (1 - frac) + (z[py1][px] * frac if frac else 0)
            cell = (px, y + sy * m)
        else:
            py, px0, px1 = y + sy * k, x + sx * q, x + sx * (q + 1)
            terr = z[py][px0] * (1 - frac) + (z[py][px1] * frac if frac else 0)
            cell = (x + sx * m, py)
        # distance along the ray is proportional to k
        s_terr = (terr - E) / k
        s_tgt = (terr + h_r - E) / k
        vis = horizon is None or s_tgt >= horizon
        if vis:
            out.add(cell)
        if dump is not None:
            dump.append((k, frac, cell, vis))
        if horizon is None or s_terr > horizon:
            horizon = s_terr
    return out


def viewshed(z, ob):
    """Set of visible cells of observer ob=(x, y, R, h_t, h_r)."""
    nrows, ncols = len(z), len(z[0])
    x, y, R = ob[0], ob[1], ob[2]
    x0, x1, y0, y1 = window(nrows, ncols, x, y, R)
    vis = {(x, y)}
    for by in range(y0, y1 + 1):
        for bx in range(x0, x1 + 1):
            if (bx in (x0, x1) or by in (y0, y1)) and (bx, by) != (x, y):
                vis |= ray(z, nrows, ncols, ob, bx, by)
    return vis


def disk(nrows, ncols, x, y, R):
    return {(cx, cy) for cy in range(max(0, y - R), min(nrows, y + R + 1))
            for cx in range(max(0, x - R), min(ncols, x + R + 1))
            if (cx - x) ** 2 + (cy - y) ** 2 <= R * R}


def greedy_sets(sets, max_obs, target):
    """Greedy maximum coverage on Python sets, ties to the lowest index."""
    cov = set()
    sel, gains = [], []
    while len(sel) < max_obs and len(cov) < target:
        best, bg = -1, -1
        for i, s in enumerate(sets):
            g = len(s - cov)
            if g > bg:
                best, bg = i, g
        if bg <= 0:
            break
        sel.append(best)
        gains.append(bg)
        cov |= sets[best]
    return sel, gains, cov


def greedy_sets_intervisible(sets, posts, max_obs, target):
    """The same greedy with intervisibility: after the first pick, only
    candidates whose post (x, y) is already covered compete."""
    cov = set()
    sel, gains = [], []
    while len(sel) < max_obs and len(cov) < target:
        best, bg = -1, -1
        for i, s in enumerate(sets):
            if sel and posts[i] not in cov:
                continue
            g = len(s - cov)
            if g > bg:
                best, bg = i, g
        if bg <= 0:
            break
        sel.append(best)
        gains.append(bg)
        cov |= sets[best]
    return sel, gains, cov


def best_cover(sets, m):
    """Exhaustive optimum coverage with m sets (tiny inputs only)."""
    best = 0
    for comb in combinations(range(len(sets)), m):
        u = set()
        for i in comb:
            u |= sets[i]
        best = max(best, len(u))
    return best


def bitmap_to_set(bm, nrows, ncols, ob):
    """Cells set in an oracle/HIP window bitmap (rows x words uint64)."""
    x, y, R = ob[0], ob[1], ob[2]
    x0, x1, y0, y1 = window(nrows, ncols, x, y, R)
    w0 = x0 >> 6
    out = set()
    for r in range(bm.shape[0]):
        for w in range(bm.shape[1]):
            v = int(bm[r, w])
            while v:
                b = (v & -v).bit_length() - 1
                out.add(((w0 + w) * 64 + b, y0 + r))
                v &= v - 1
    return out
