/*
 * oracle.c -- plain, slow CPU oracle for the multiple-observer siting method
 * (Franklin, Magalhaes, Li: "Siting thousands of radio transmitter towers on
 * terrains with billions of points", arXiv 2006.16783).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links or calls this
 * file; only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark do.  It shares no code, header, table or constant generator with
 * the HIP library: every definition below is written out again from the paper
 * (and from the published definition of the Philox generator).
 *
 * Integer work throughout: every comparison is exact, so the HIP path must
 * match this file bit for bit.
 *
 * Readings of the paper that this file fixes (the paper is silent on them):
 *  - frame: x = column, y = row, posts one unit apart; observer eye at
 *    z[T] + h_t, receiver top at z[P] + h_r (section "Terrain visibility");
 *  - line of sight samples the terrain where the segment crosses grid lines
 *    of the major axis, linearly interpolated between the two adjacent posts;
 *    the target is blocked only if the terrain is strictly above the segment
 *    (tangency is visible);
 *  - VIX targets are uniform over the lattice cells of the ROI disk that lie
 *    inside the terrain, drawn by rejection from the terrain-clipped bounding
 *    box with one counter-based Philox4x32-10 stream per post;
 *  - FINDMAX blocks are a G_r x G_c grid with floor(i*N/G) boundaries, ranked
 *    by (count desc, elevation desc, linear index asc);
 *  - the viewshed sweeps rays from the observer to every boundary cell of the
 *    terrain-clipped (2R+1)^2 window, marks at each major-axis step the cell
 *    nearest to the ray (ties away from the observer), stops when that cell
 *    leaves the ROI disk, and keeps a horizon of terrain slopes compared by
 *    exact cross-multiplication;
 *  - SITE is greedy maximum coverage with ties to the lowest candidate index.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int32_t x, y, roi, h_t, h_r;
} or_observer;

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11 "Parallel random numbers:
 * as easy as 1, 2, 3").  Each round multiplies counter words 0 and 2 by the
 * round multipliers into 64-bit products; the high halves are mixed with the
 * other two words and the key, the low halves move to words 1 and 3, and the
 * key is bumped by the Weyl constants between rounds.                       */
void or_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t x0 = ctr_in[0], x1 = ctr_in[1], x2 = ctr_in[2], x3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; round++) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * x2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        x0 = n0; x1 = n1; x2 = n2; x3 = n3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* ------------------------------------------------------------------------ */
/* Terrain access: z is row-major with leading dimension ld (posts per row). */
static inline int64_t Z(const int16_t *z, int64_t ld, int64_t x, int64_t y)
{
    return (int64_t)z[y * ld + x];
}

/* Line of sight between observer T=(tx,ty) and receiver P=(px,py).
 * Returns 1 if P is visible.  Definitions section (line of sight) and the
 * "Terrain visibility" section (linear interpolation between adjacent
 * posts).  All arithmetic is exact in int64: at major step k the segment
 * crosses the grid line at minor offset k*|minor|/n = q + r/n, the terrain
 * there is (z0*(n-r) + z1*r)/n, and the segment height is E + (Z-E)*k/n.   */
int or_los(const int16_t *z, int64_t nrows, int64_t ncols, int64_t ld,
           int64_t tx, int64_t ty, int64_t px, int64_t py, int32_t h_t, int32_t h_r)
{
    (void)nrows; (void)ncols;
    int64_t dx = px - tx, dy = py - ty;
    int64_t adx = dx < 0 ? -dx : dx, ady = dy < 0 ? -dy : dy;
    int64_t sx = dx < 0 ? -1 : 1, sy = dy < 0 ? -1 : 1;
    int xmajor = adx >= ady;
    int64_t n = xmajor ? adx : ady;
    int64_t mn = xmajor ? ady : adx;
    if (n <= 1)
        return 1;
    int64_t E = Z(z, ld, tx, ty) + h_t;
    int64_t Zt = Z(z, ld, px, py) + h_r;
    for (int64_t k = 1; k <= n - 1; k++) {
        int64_t q = (k * mn) / n;
        int64_t r = (k * mn) % n;
        int64_t x0, y0, x1, y1;
        if (xmajor) {
            x0 = tx + sx * k; y0 = ty + sy * q;
            x1 = x0;          y1 = ty + sy * (q + 1);
        } else {
            y0 = ty + sy * k; x0 = tx + sx * q;
            y1 = y0;          x1 = tx + sx * (q + 1);
        }
        int64_t z0 = Z(z, ld, x0, y0);
        int64_t z1 = r > 0 ? Z(z, ld, x1, y1) : 0;
        int64_t S = z0 * (n - r) + z1 * r;
        if (S > E * n + (Zt - E) * k)
            return 0;
    }
    return 1;
}

/* ------------------------------------------------------------------------ */
/* VIX (section "The multiple transmitter siting process", stage Vix):
 * for every post, K receivers drawn uniformly from the ROI disk, each tested
 * for line of sight; the output is the number of visible receivers.
 *
 * Post t (t = y*ncols + x) owns one stream of 32-bit words: word a is word
 * (a mod 4) of Philox4x32-10(counter = {t mod 2^32, a/4, t / 2^32, 0},
 * key = {seed mod 2^32, seed / 2^32}).  Each word u makes one proposal in
 * the terrain-clipped box [bx0, bx0+wx) x [by0, by0+wy) around the post: its
 * low and high 16 bits fx, fy are scaled to the box widths by Lemire's
 * multiply-shift with rejection (Lemire, "Fast random integer generation in
 * an interval", ACM TOMACS 2019):
 *     mx = fx * wx,  accepted only if (mx mod 2^16) >= 2^16 mod wx,
 *     px = bx0 + mx / 2^16,
 * and the same for y, which makes (px, py) exactly uniform over the box.
 * The proposal is accepted iff both scalings accept, (px,py) != (x,y) and
 * (px-x)^2 + (py-y)^2 <= R^2.  Draw j is the next accepted proposal; after 64
 * consecutive rejections draw j fails (counts as not visible) and draw j+1
 * continues with the following word.  The K targets of post (x,y) can be
 * dumped with or_vix_targets.                                              */
#define OR_VIX_MAX_ATTEMPTS 64

typedef struct {
    int64_t t, x, y, bx0, by0;
    uint64_t wx, wy, seed;
    uint64_t a;          /* next word of the stream */
    uint32_t blk[4];
} vix_stream;

static void vix_stream_init(vix_stream *s, int64_t nrows, int64_t ncols, int64_t x, int64_t y,
                            int32_t R, uint64_t seed)
{
    s->t = y * ncols + x;
    s->x = x; s->y = y;
    s->bx0 = x - R < 0 ? 0 : x - R;
    int64_t bx1 = x + R > ncols - 1 ? ncols - 1 : x + R;
    s->by0 = y - R < 0 ? 0 : y - R;
    int64_t by1 = y + R > nrows - 1 ? nrows - 1 : y + R;
    s->wx = (uint64_t)(bx1 - s->bx0 + 1);
    s->wy = (uint64_t)(by1 - s->by0 + 1);
    s->seed = seed;
    s->a = 0;
}

/* Lemire's bounded integer from a 16-bit field f: 1 and *v in [0, w), or 0
 * when the field falls in the rejected sliver. */
static int lemire16(uint64_t f, uint64_t w, int64_t *v)
{
    uint64_t m = f * w;
    if ((m & 0xffff) < (65536 % w))
        return 0;
    *v = (int64_t)(m >> 16);
    return 1;
}

static int vix_draw(vix_stream *s, int32_t R, int64_t *ox, int64_t *oy)
{
    uint32_t key[2] = {(uint32_t)s->seed, (uint32_t)(s->seed >> 32)};
    for (int att = 0; att < OR_VIX_MAX_ATTEMPTS; att++) {
        if ((s->a & 3) == 0) {
            uint32_t ctr[4] = {(uint32_t)s->t, (uint32_t)(s->a >> 2),
                               (uint32_t)((uint64_t)s->t >> 32), 0};
            or_philox4x32_10(ctr, key, s->blk);
        }
        uint64_t u = s->blk[s->a & 3];
        s->a++;
        int64_t ox_, oy_;
        if (!lemire16(u & 0xffff, s->wx, &ox_) || !lemire16(u >> 16, s->wy, &oy_))
            continue;
        int64_t px = s->bx0 + ox_, py = s->by0 + oy_;
        int64_t ddx = px - s->x, ddy = py - s->y;
        if ((ddx != 0 || ddy != 0) && ddx * ddx + ddy * ddy <= (int64_t)R * R) {
            *ox = px; *oy = py;
            return 1;
        }
    }
    return 0;
}

/* The count of one post: K draws, each tested for line of sight. */
static uint8_t vix_post(const int16_t *z, int64_t nrows, int64_t ncols, int64_t ld, int64_t x,
                        int64_t y, int32_t R, int32_t h_t, int32_t h_r, int32_t K, uint64_t seed)
{
    int c = 0;
    vix_stream st;
    vix_stream_init(&st, nrows, ncols, x, y, R, seed);
    for (int32_t j = 0; j < K; j++) {
        int64_t px, py;
        if (vix_draw(&st, R, &px, &py))
            c += or_los(z, nrows, ncols, ld, x, y, px, py, h_t, h_r);
    }
    return (uint8_t)c;
}

/* Rows [row0,row1) of the count array (the full terrain when row0=0,
 * row1=nrows); count has nrows x ncols entries, row-major, contiguous.     */
void or_vix(const int16_t *z, int64_t nrows, int64_t ncols, int64_t ld,
            int32_t R, int32_t h_t, int32_t h_r, int32_t K, uint64_t seed,
            uint8_t *count, int64_t row0, int64_t row1)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t y = row0; y < row1; y++)
        for (int64_t x = 0; x < ncols; x++)
            count[y * ncols + x] = vix_post(z, nrows, ncols, ld, x, y, R, h_t, h_r, K, seed);
}

/* The counts of the posts of rows rows[0..nlist) only, into count_rows
 * (nlist x ncols, row-major); the work is split into chunks of columns so
 * that a short list of long rows still spreads over the threads.           */
void or_vix_rowlist(const int16_t *z, int64_t nrows, int64_t ncols, int64_t ld,
                    int32_t R, int32_t h_t, int32_t h_r, int32_t K, uint64_t seed,
                    const int64_t *rows, int64_t nlist, uint8_t *count_rows)
{
    const int64_t chunk = 4096, nch = (ncols + chunk - 1) / chunk;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t w = 0; w < nlist * nch; w++) {
        int64_t i = w / nch, x0 = (w % nch) * chunk;
        int64_t x1 = x0 + chunk < ncols ? x0 + chunk : ncols;
        for (int64_t x = x0; x < x1; x++)
            count_rows[i * ncols + x] = vix_post(z, nrows, ncols, ld, x, rows[i], R, h_t, h_r, K,
                                                 seed);
    }
}

/* The K targets of one post (for tests): tx/ty get -1 for a failed draw. */
void or_vix_targets(int64_t nrows, int64_t ncols, int64_t x, int64_t y, int32_t R,
                    int32_t K, uint64_t seed, int64_t *tx, int64_t *ty)
{
    vix_stream st;
    vix_stream_init(&st, nrows, ncols, x, y, R, seed);
    for (int32_t j = 0; j < K; j++) {
        int64_t px = -1, py = -1;
        vix_draw(&st, R, &px, &py);
        tx[j] = px; ty[j] = py;
    }
}

/* ------------------------------------------------------------------------ */
/* FINDMAX (stage Findmax): split the terrain into a grid_r x grid_c grid of
 * blocks with boundaries floor(i*N/G) and keep, per block, the k best posts.
 * Blocks are output in row-major order, each with k slots, best first,
 * padded with -1 when the block has fewer than k posts.                     */
typedef struct {
    double key;      /* primary key, larger is better */
    int64_t z;       /* elevation, larger is better (u8 keys only) */
    int64_t idx;     /* linear post index y*ncols+x, smaller is better */
} fm_item;

static int fm_cmp(const void *pa, const void *pb)
{
    const fm_item *a = (const fm_item *)pa, *b = (const fm_item *)pb;
    if (a->key != b->key) return a->key > b->key ? -1 : 1;
    if (a->z != b->z) return a->z > b->z ? -1 : 1;
    if (a->idx != b->idx) return a->idx < b->idx ? -1 : 1;
    return 0;
}

/* key_type 0: uint8 keys (VIX counts), one per post; rank (key desc, z desc,
 * index asc).  key_type 1: float keys (surrogate scores) of the cells of a
 * stride x stride grid (key array of ceil(nrows/stride) x ceil(ncols/stride));
 * a cell belongs to the block holding its corner post (i*stride, j*stride),
 * ranks by (key desc, cell index asc) with NaN as -infinity, and stands for
 * its highest post (elevation desc, index asc), which is the candidate
 * returned.                                                               */
int64_t or_cell_max(const int16_t *z, int64_t nrows, int64_t ncols, int64_t ld, int32_t stride,
                    int64_t ci, int64_t cj)
{
    int64_t best = -1, bz = 0;
    for (int64_t y = ci * stride; y < (ci + 1) * stride && y < nrows; y++)
        for (int64_t x = cj * stride; x < (cj + 1) * stride && x < ncols; x++) {
            int64_t v = Z(z, ld, x, y);
            if (best < 0 || v > bz) {
                best = y * ncols + x;
                bz = v;
            }
        }
    return best;
}

void or_findmax(const void *key, int32_t key_type, int32_t stride,
                const int16_t *z, int64_t nrows, int64_t ncols, int64_t ld,
                int32_t grid_r, int32_t grid_c, int32_t k, int64_t *cand)
{
    int64_t kc = (ncols + stride - 1) / stride;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t b = 0; b < (int64_t)grid_r * grid_c; b++) {
        int64_t bi = b / grid_c, bj = b % grid_c;
        int64_t r0 = bi * nrows / grid_r, r1 = (bi + 1) * nrows / grid_r;
        int64_t c0 = bj * ncols / grid_c, c1 = (bj + 1) * ncols / grid_c;
        int64_t cap = (r1 - r0) * (c1 - c0);
        fm_item *items = (fm_item *)malloc((size_t)(cap > 0 ? cap : 1) * sizeof(fm_item));
        int64_t m = 0;
        for (int64_t y = r0; y < r1; y++)
            for (int64_t x = c0; x < c1; x++) {
                fm_item it;
                it.idx = y * ncols + x;
                if (key_type == 0) {
                    it.key = (double)((const uint8_t *)key)[y * ncols + x];
                    it.z = Z(z, ld, x, y);
                } else {
                    if (y % stride || x % stride) continue;
                    float f = ((const float *)key)[(y / stride) * kc + (x / stride)];
                    it.key = (f != f) ? -1.0 / 0.0 : (double)f;
                    it.z = 0;
                }
                items[m++] = it;
            }
        qsort(items, (size_t)m, sizeof(fm_item), fm_cmp);
        for (int32_t i = 0; i < k; i++) {
            int64_t c = i < m ? items[i].idx : -1;
            if (c >= 0 && key_type == 1)
                c = or_cell_max(z, nrows, ncols, ld, stride, (c / ncols) / stride,
                                (c % ncols) / stride);
            cand[b * k + i] = c;
        }
        free(items);
    }
}

/* ------------------------------------------------------------------------ */
/* Viewshed window geometry (stage Viewshed; bitmaps in 64-bit words):
 * rows [max(0,y-R), min(nrows-1,y+R)], words [max(0,x-R)>>6,
 * min(ncols-1,x+R)>>6]; bit (c & 63) of word (c >> 6) is global column c.  */
static void window(const or_observer *o, int64_t nrows, int64_t ncols,
                   int64_t *xlo, int64_t *xhi, int64_t *ylo, int64_t *yhi,
                   int64_t *w0, int64_t *nw)
{
    int64_t R = o->roi;
    *xlo = o->x - R < 0 ? 0 : o->x - R;
    *xhi = o->x + R > ncols - 1 ? ncols - 1 : o->x + R;
    *ylo = o->y - R < 0 ? 0 : o->y - R;
    *yhi = o->y + R > nrows - 1 ? nrows - 1 : o->y + R;
    *w0 = *xlo >> 6;
    *nw = (*xhi >> 6) - *w0 + 1;
}

/* offsets[i] = first word of observer i's window bitmap; offsets[n] = total */
int64_t or_layout(const or_observer *obs, int64_t n, int64_t nrows, int64_t ncols,
                  int64_t *offsets)
{
    int64_t off = 0;
    for (int64_t i = 0; i < n; i++) {
        int64_t xlo, xhi, ylo, yhi, w0, nw;
        window(&obs[i], nrows, ncols, &xlo, &xhi, &ylo, &yhi, &w0, &nw);
        offsets[i] = off;
        off += (yhi - ylo + 1) * nw;
    }
    offsets[n] = off;
    return off;
}

static inline void setbit(uint64_t *bm, int64_t nw, int64_t w0, int64_t ylo,
                          int64_t x, int64_t y)
{
    int64_t w = (y - ylo) * nw + ((x >> 6) - w0);
    bm[w] |= 1ULL << (x & 63);
}

/* One ray from T to boundary cell B (stage Viewshed: walk along the line of
 * sight updating a horizon).  At major step k (k*|minor| = q*n + r):
 *   S_k = z0*(n-r) + z1*r is n times the interpolated terrain on the crossed
 *       grid line (z0 at minor q, z1 at minor q+1);
 *   the marked cell is at minor q + [2r >= n] (nearest, ties away from T);
 *   the ray stops when the marked cell leaves the ROI disk;
 *   with horizon (S_J, J), the cell is visible iff the slope of the terrain
 *       plus h_r, (S_k + h_r*n - E*n)/k, is >= the horizon slope
 *       (S_J - E*n)/J, compared as (S_k + h_r n - E n) J >= (S_J - E n) k;
 *   then the horizon moves to (S_k, k) iff (S_k - E n) J > (S_J - E n) k.
 * The first step has no horizon: its cell is visible and sets the horizon. */
static void sweep_ray(const int16_t *z, int64_t ld, const or_observer *o,
                      int64_t bx, int64_t by, uint64_t *bm, int64_t nw,
                      int64_t w0, int64_t ylo)
{
    int64_t tx = o->x, ty = o->y, R = o->roi;
    int64_t dx = bx - tx, dy = by - ty;
    int64_t adx = dx < 0 ? -dx : dx, ady = dy < 0 ? -dy : dy;
    int64_t sx = dx < 0 ? -1 : 1, sy = dy < 0 ? -1 : 1;
    int xmajor = adx >= ady;
    int64_t n = xmajor ? adx : ady;
    int64_t mn = xmajor ? ady : adx;
    int64_t E = Z(z, ld, tx, ty) + o->h_t;
    int64_t En = E * n, hrn = (int64_t)o->h_r * n;
    int have_horizon = 0;
    int64_t SJ = 0, J = 0;
    for (int64_t k = 1; k <= n; k++) {
        int64_t q = (k * mn) / n, r = (k * mn) % n;
        int64_t m = q + (2 * r >= n ? 1 : 0);
        if (k * k + m * m > R * R)
            break;
        int64_t x0, y0, x1, y1, mx, my;
        if (xmajor) {
            x0 = tx + sx * k; y0 = ty + sy * q; x1 = x0; y1 = ty + sy * (q + 1);
            mx = x0;          my = ty + sy * m;
        } else {
            y0 = ty + sy * k; x0 = tx + sx * q; y1 = y0; x1 = tx + sx * (q + 1);
            my = y0;          mx = tx + sx * m;
        }
        int64_t z0 = Z(z, ld, x0, y0);
        int64_t z1 = r > 0 ? Z(z, ld, x1, y1) : 0;
        int64_t S = z0 * (n - r) + z1 * r;
        int visible, raise;
        if (!have_horizon) {
            visible = 1;
            raise = 1;
        } else {
            visible = (S + hrn - En) * J >= (SJ - En) * k;
            raise = (S - En) * J > (SJ - En) * k;
        }
        if (visible)
            setbit(bm, nw, w0, ylo, mx, my);
        if (raise) {
            SJ = S; J = k; have_horizon = 1;
        }
    }
}

/* Viewshed of one observer into its window bitmap (zeroed here). */
void or_viewshed_one(const int16_t *z, int64_t nrows, int64_t ncols, int64_t ld,
                     const or_observer *o, uint64_t *bm)
{
    int64_t xlo, xhi, ylo, yhi, w0, nw;
    window(o, nrows, ncols, &xlo, &xhi, &ylo, &yhi, &w0, &nw);
    memset(bm, 0, (size_t)((yhi - ylo + 1) * nw) * sizeof(uint64_t));
    setbit(bm, nw, w0, ylo, o->x, o->y);
    for (int64_t by = ylo; by <= yhi; by++)
        for (int64_t bx = xlo; bx <= xhi; bx++) {
            int on_boundary = bx == xlo || bx == xhi || by == ylo || by == yhi;
            if (!on_boundary || (bx == o->x && by == o->y))
                continue;
            sweep_ray(z, ld, o, bx, by, bm, nw, w0, ylo);
        }
}

/* Viewsheds of observers [i0,i1) into bitmaps at their layout offsets. */
void or_viewshed(const int16_t *z, int64_t nrows, int64_t ncols, int64_t ld,
                 const or_observer *obs, const int64_t *offsets, int64_t i0, int64_t i1,
                 uint64_t *bitmaps)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = i0; i < i1; i++)
        or_viewshed_one(z, nrows, ncols, ld, &obs[i], bitmaps + offsets[i]);
}

/* Exact per-cell viewshed (the R3 family the paper cites as prior art for
 * viewsheds, and the definition the ray sweep approximates): every lattice
 * cell P of the ROI disk inside the terrain is visible iff the line of sight
 * from the observer to P is clear (or_los above); the observer's own cell is
 * visible.  Same window layout as or_viewshed_one.                         */
void or_viewshed_r3_one(const int16_t *z, int64_t nrows, int64_t ncols, int64_t ld,
                        const or_observer *o, uint64_t *bm)
{
    int64_t xlo, xhi, ylo, yhi, w0, nw;
    window(o, nrows, ncols, &xlo, &xhi, &ylo, &yhi, &w0, &nw);
    memset(bm, 0, (size_t)((yhi - ylo + 1) * nw) * sizeof(uint64_t));
    int64_t R = o->roi;
    for (int64_t py = ylo; py <= yhi; py++)
        for (int64_t px = xlo; px <= xhi; px++) {
            int64_t dx = px - o->x, dy = py - o->y;
            if (dx * dx + dy * dy > R * R)
                continue;
            if (or_los(z, nrows, ncols, ld, o->x, o->y, px, py, o->h_t, o->h_r))
                setbit(bm, nw, w0, ylo, px, py);
        }
}

void or_viewshed_r3(const int16_t *z, int64_t nrows, int64_t ncols, int64_t ld,
                    const or_observer *obs, const int64_t *offsets, int64_t i0, int64_t i1,
                    uint64_t *bitmaps)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = i0; i < i1; i++)
        or_viewshed_r3_one(z, nrows, ncols, ld, &obs[i], bitmaps + offsets[i]);
}

/* Number of lattice cells of observer o's ROI disk inside the terrain. */
int64_t or_disk_cells(const or_observer *o, int64_t nrows, int64_t ncols)
{
    int64_t c = 0, R = o->roi;
    for (int64_t y = o->y - R; y <= o->y + R; y++)
        for (int64_t x = o->x - R; x <= o->x + R; x++) {
            int64_t dx = x - o->x, dy = y - o->y;
            if (x < 0 || y < 0 || x >= ncols || y >= nrows) continue;
            if (dx * dx + dy * dy <= R * R) c++;
        }
    return c;
}

/* Visible-cell count and disk-cell count per observer (visibility index
 * numerator and denominator, Definitions section).                        */
void or_viewshed_count(const int16_t *z, int64_t nrows, int64_t ncols, int64_t ld,
                       const or_observer *obs, int64_t n, uint32_t *visible, uint32_t *cells)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < n; i++) {
        int64_t xlo, xhi, ylo, yhi, w0, nw;
        window(&obs[i], nrows, ncols, &xlo, &xhi, &ylo, &yhi, &w0, &nw);
        int64_t words = (yhi - ylo + 1) * nw;
        uint64_t *bm = (uint64_t *)malloc((size_t)words * sizeof(uint64_t));
        or_viewshed_one(z, nrows, ncols, ld, &obs[i], bm);
        int64_t v = 0;
        for (int64_t w = 0; w < words; w++)
            v += __builtin_popcountll(bm[w]);
        free(bm);
        visible[i] = (uint32_t)v;
        cells[i] = (uint32_t)or_disk_cells(&obs[i], nrows, ncols);
    }
}

/* ------------------------------------------------------------------------ */
/* SITE (stage Site): greedy maximum coverage over the candidate viewsheds.
 * gain_i = |V_i \ C|; the winner is the largest gain, ties to the smallest
 * candidate index; stop at max_obs observers, when |C| >= target_cells, or
 * when the best gain is 0.  cumulative has nrows x ceil(ncols/64) words and
 * is zeroed here.  Returns the number selected.                            */
static int64_t gain_of(const uint64_t *bitmaps, const int64_t *offsets, const or_observer *o,
                       int64_t i, int64_t nrows, int64_t ncols, const uint64_t *C, int64_t W)
{
    int64_t xlo, xhi, ylo, yhi, w0, nw;
    window(o, nrows, ncols, &xlo, &xhi, &ylo, &yhi, &w0, &nw);
    const uint64_t *v = bitmaps + offsets[i];
    int64_t g = 0;
    for (int64_t y = ylo; y <= yhi; y++)
        for (int64_t w = 0; w < nw; w++)
            g += __builtin_popcountll(v[(y - ylo) * nw + w] & ~C[y * W + w0 + w]);
    return g;
}

static void unite(const uint64_t *bitmaps, const int64_t *offsets, const or_observer *o,
                  int64_t i, int64_t nrows, int64_t ncols, uint64_t *C, int64_t W)
{
    int64_t xlo, xhi, ylo, yhi, w0, nw;
    window(o, nrows, ncols, &xlo, &xhi, &ylo, &yhi, &w0, &nw);
    const uint64_t *v = bitmaps + offsets[i];
    for (int64_t y = ylo; y <= yhi; y++)
        for (int64_t w = 0; w < nw; w++)
            C[y * W + w0 + w] |= v[(y - ylo) * nw + w];
}

/* Intervisibility (a constraint the paper names among the variants of the
 * problem: transmitters must be visible from other transmitters).  Read as:
 * after the first selection, a candidate may be selected only if its own
 * post lies in the cumulative viewshed of those already selected, i.e. it
 * is visible from at least one of them; the first selection is free.  A
 * candidate outside the terrain is never eligible after the first round.  */
static int eligible(const or_observer *o, int64_t nrows, int64_t ncols, const uint64_t *C,
                    int64_t W, int32_t t)
{
    if (t == 0)
        return 1;
    if (o->x < 0 || o->x >= ncols || o->y < 0 || o->y >= nrows)
        return 0;
    return (int)((C[(int64_t)o->y * W + (o->x >> 6)] >> (o->x & 63)) & 1u);
}

/* inter != 0: only eligible candidates (above) compete in each round; the
 * run stops when no eligible candidate gains anything.                    */
int32_t or_greedy(const uint64_t *bitmaps, const int64_t *offsets, const or_observer *obs,
                  int64_t n, int64_t nrows, int64_t ncols, int32_t max_obs, int64_t target_cells,
                  uint64_t *cumulative, int64_t *selected, int64_t *gains, int32_t inter)
{
    int64_t W = (ncols + 63) / 64;
    memset(cumulative, 0, (size_t)(nrows * W) * sizeof(uint64_t));
    int64_t *g = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    int64_t covered = 0;
    int32_t t = 0;
    while (t < max_obs && covered < target_cells) {
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t i = 0; i < n; i++)
            g[i] = gain_of(bitmaps, offsets, &obs[i], i, nrows, ncols, cumulative, W);
        int64_t best = -1;
        for (int64_t i = 0; i < n; i++)
            if ((!inter || eligible(&obs[i], nrows, ncols, cumulative, W, t)) &&
                (best < 0 || g[i] > g[best]))
                best = i;
        if (best < 0 || g[best] == 0)
            break;
        selected[t] = best;
        gains[t] = g[best];
        covered += g[best];
        unite(bitmaps, offsets, &obs[best], best, nrows, ncols, cumulative, W);
        t++;
    }
    free(g);
    return t;
}

/* The same selection with the paper's optimisation that a candidate's gain
 * can only shrink as the cumulative viewshed grows (lazy evaluation, Minoux's
 * accelerated greedy): the stale gains are upper bounds; the candidate with
 * the largest bound (ties to the smallest index) is re-evaluated, and is
 * taken once its bound is fresh for the current round.  Same tie rule, so
 * the same selection as or_greedy (with or without intervisibility).      */
int32_t or_greedy_lazy(const uint64_t *bitmaps, const int64_t *offsets, const or_observer *obs,
                       int64_t n, int64_t nrows, int64_t ncols, int32_t max_obs,
                       int64_t target_cells, uint64_t *cumulative, int64_t *selected,
                       int64_t *gains, int64_t *n_evals, int32_t inter)
{
    int64_t W = (ncols + 63) / 64;
    memset(cumulative, 0, (size_t)(nrows * W) * sizeof(uint64_t));
    int64_t *bound = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    int32_t *fresh = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    for (int64_t i = 0; i < n; i++) {
        bound[i] = gain_of(bitmaps, offsets, &obs[i], i, nrows, ncols, cumulative, W);
        fresh[i] = 0;
    }
    int64_t evals = n, covered = 0;
    int32_t t = 0;
    while (t < max_obs && covered < target_cells && n > 0) {
        /* with intervisibility, the bounds of the eligible candidates only
         * (a bound stays valid while a candidate waits to become eligible) */
        int64_t best = -1;
        for (int64_t i = 0; i < n; i++)
            if ((!inter || eligible(&obs[i], nrows, ncols, cumulative, W, t)) &&
                (best < 0 || bound[i] > bound[best]))
                best = i;
        if (best < 0)
            break;
        if (fresh[best] != t) {
            bound[best] = gain_of(bitmaps, offsets, &obs[best], best, nrows, ncols, cumulative, W);
            fresh[best] = t;
            evals++;
            continue;
        }
        if (bound[best] == 0)
            break;
        selected[t] = best;
        gains[t] = bound[best];
        covered += bound[best];
        unite(bitmaps, offsets, &obs[best], best, nrows, ncols, cumulative, W);
        bound[best] = 0;
        t++;
        fresh[best] = t;
    }
    if (n_evals) *n_evals = evals;
    free(bound);
    free(fresh);
    return t;
}

int32_t or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads for the parallel loops above (timing only; results do not depend
 * on it): n >= 1. */
void or_set_threads(int32_t n)
{
#ifdef _OPENMP
    omp_set_num_threads(n > 0 ? n : 1);
#else
    (void)n;
#endif
}
