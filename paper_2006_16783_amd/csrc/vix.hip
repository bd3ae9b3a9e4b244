// VIX: estimated visibility index of every post from K random receivers in
// its ROI disk (stage Vix of the siting process), one lane per post.
//
// Layout: the terrain is cut into T x T post tiles; a workgroup stages its
// tile plus an R-post halo ((T+2R)^2 int16) in LDS when that fits, so every
// line-of-sight sample is an LDS read; otherwise (large ROI) it reads the
// terrain through L2 and tiles only give spatial locality.  Tiles are handed
// to XCDs in contiguous bands so that neighbouring halos share an L2.
//
// Exactness: everything is integer.  At major step k of a LOS of length n
// (k*|minor| = q*n + r) the terrain sample is S = z0*n + (z1-z0)*r and the
// segment is E*n + (Z-E)*k; with |z| < 2^15, n <= 16383 and heights <= 2^15
// every term fits in int32 and the 24-bit multiplier is exact.
#include "common.hpp"

namespace siting {
namespace {

constexpr int kVixThreads = 1024;
constexpr int kVixMaxAttempts = 64;

// Philox4x64-10 block function (Salmon et al., SC'11).
__device__ __forceinline__ void philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                              uint64_t k0, uint64_t k1, uint64_t out[4])
{
    constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int round = 0; round < 10; round++) {
        uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
        uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
        uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += W0; k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

// Terrain accessor: LDS tile (int16 in shared memory) or global memory.
struct LdsTerrain {
    const int16_t *base;  // LDS tile; (gx, gy) at (gy - oy) * pitch + (gx - ox)
    int pitch;
    int64_t ox, oy;
    __device__ __forceinline__ int offset(int64_t gx, int64_t gy) const
    {
        return (int)((gy - oy) * pitch + (gx - ox));
    }
    __device__ __forceinline__ int row_stride() const { return pitch; }
    __device__ __forceinline__ int at(int off) const { return base[off]; }
};

struct GlobalTerrain {
    const int16_t *base;  // global terrain; (gx, gy) at gy * ld + gx, relative to the post
    int64_t ld;
    __device__ __forceinline__ int row_stride() const { return (int)ld; }
    __device__ __forceinline__ int at(int off) const { return base[off]; }
};

// One line-of-sight test.  `acc.at(0)` is the observer post; target at
// (dx, dy).  Returns 1 if the receiver is visible.
template <bool kCount, class Acc>
__device__ __forceinline__ int los(const Acc &acc, int dx, int dy, int E, int Zt, uint64_t &steps)
{
    int adx = dx < 0 ? -dx : dx, ady = dy < 0 ? -dy : dy;
    int rs = acc.row_stride();
    int sx = dx < 0 ? -1 : 1, sy = dy < 0 ? -rs : rs;
    bool xmaj = adx >= ady;
    int n = xmaj ? adx : ady, mn = xmaj ? ady : adx;
    int s_maj = xmaj ? sx : sy, s_min = xmaj ? sy : sx;
    if (n <= 1)
        return 1;
    int rhs = __mul24(E, n);
    int dz = Zt - E;
    int r = 0, off = 0;
    for (int k = 1; k < n; k++) {
        if (kCount)
            steps++;
        r += mn;
        off += s_maj;
        if (r >= n) {
            r -= n;
            off += s_min;
        }
        int z0 = acc.at(off);
        int z1 = acc.at(off + s_min);  // in the observer-target box for k < n
        int S = __mul24(z0, n) + __mul24(z1 - z0, r);
        rhs += dz;
        if (S > rhs)
            return 0;
    }
    return 1;
}

template <bool kLds, bool kCount>
__global__ __launch_bounds__(kVixThreads) void vix_kernel(
    const int16_t *__restrict__ z, int64_t nrows, int64_t ncols, int64_t ld, int R, int h_t,
    int h_r, int K, uint64_t seed, uint8_t *__restrict__ count, int T, int64_t tiles_r,
    int64_t tiles_c, int64_t per_xcd, unsigned long long *__restrict__ stats)
{
    uint64_t steps = 0, tests = 0;
    extern __shared__ int16_t tile[];
    // XCD-aware tile order: workgroup b runs on XCD b % 8; give each XCD a
    // contiguous band of tiles.
    int64_t b = blockIdx.x;
    int64_t t_id = (b & 7) * per_xcd + (b >> 3);
    if (t_id >= tiles_r * tiles_c)
        return;
    int64_t tr = t_id / tiles_c, tc = t_id % tiles_c;
    int64_t r0 = tr * T, c0 = tc * T;
    int64_t oy = r0 - R, ox = c0 - R;
    int pitch = T + 2 * R;
    if (kLds) {
        int64_t gy0 = oy < 0 ? 0 : oy, gy1 = r0 + T + R > nrows ? nrows : r0 + T + R;
        int64_t gx0 = ox < 0 ? 0 : ox, gx1 = c0 + T + R > ncols ? ncols : c0 + T + R;
        int w = (int)(gx1 - gx0), h = (int)(gy1 - gy0);
        int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nwaves = blockDim.x >> 6;
        for (int row = wave; row < h; row += nwaves) {
            const int16_t *src = z + (gy0 + row) * ld + gx0;
            int16_t *dst = tile + (gy0 + row - oy) * pitch + (gx0 - ox);
            for (int col = lane; col < w; col += 64)
                dst[col] = src[col];
        }
        __syncthreads();
    }
    int64_t tile_rows = (r0 + T > nrows ? nrows : r0 + T) - r0;
    int64_t tile_cols = (c0 + T > ncols ? ncols : c0 + T) - c0;
    int64_t R2 = (int64_t)R * R;
    for (int p = threadIdx.x; p < T * T; p += blockDim.x) {
        int py = p / T, px = p % T;
        if (py >= tile_rows || px >= tile_cols)
            continue;
        int64_t y = r0 + py, x = c0 + px;
        int64_t t = y * ncols + x;
        int64_t bx0 = x - R < 0 ? 0 : x - R, bx1 = x + R > ncols - 1 ? ncols - 1 : x + R;
        int64_t by0 = y - R < 0 ? 0 : y - R, by1 = y + R > nrows - 1 ? nrows - 1 : y + R;
        uint64_t wx = (uint64_t)(bx1 - bx0 + 1), wy = (uint64_t)(by1 - by0 + 1);
        int E, cnt = 0;
        LdsTerrain la;
        GlobalTerrain ga;
        if (kLds) {
            la.pitch = pitch; la.ox = ox; la.oy = oy;
            la.base = tile + la.offset(x, y);
            E = la.at(0) + h_t;
        } else {
            ga.base = z + y * ld + x;
            ga.ld = ld;
            E = ga.at(0) + h_t;
        }
        for (int j = 0; j < K; j++) {
            uint64_t blk[4];
            int dx = 0, dy = 0, ok = 0;
            for (int a = 0; a < kVixMaxAttempts && !ok; a++) {
                if ((a & 3) == 0)
                    philox4x64_10((uint64_t)t, (uint64_t)j, (uint64_t)(a >> 2), 0, seed, 0, blk);
                uint64_t u = blk[a & 3];
                int64_t px_ = bx0 + (int64_t)(((u >> 32) * wx) >> 32);
                int64_t py_ = by0 + (int64_t)(((u & 0xffffffffull) * wy) >> 32);
                int64_t ddx = px_ - x, ddy = py_ - y;
                if ((ddx | ddy) != 0 && ddx * ddx + ddy * ddy <= R2) {
                    ok = 1;
                    dx = (int)ddx;
                    dy = (int)ddy;
                }
            }
            if (!ok)
                continue;
            if (kCount)
                tests++;
            if (kLds) {
                int Zt = la.at(dy * pitch + dx) + h_r;
                cnt += los<kCount>(la, dx, dy, E, Zt, steps);
            } else {
                int Zt = ga.at((int)(dy * ld + dx)) + h_r;
                cnt += los<kCount>(ga, dx, dy, E, Zt, steps);
            }
        }
        count[t] = (uint8_t)cnt;
    }
    if (kCount) {
        // per-lane totals; the one global atomic per lane is negligible next
        // to the line-of-sight work and only runs in this counting variant
        atomicAdd(&stats[0], (unsigned long long)steps);
        atomicAdd(&stats[1], (unsigned long long)tests);
    }
}

__global__ void vix_stats_reset(unsigned long long *stats)
{
    stats[0] = 0;
    stats[1] = 0;
}

}  // namespace
}  // namespace siting

using namespace siting;

static int vix_launch(const int16_t *z, int64_t nrows, int64_t ncols, int64_t ld, int32_t roi,
                      int32_t h_t, int32_t h_r, int32_t K, uint64_t seed, uint8_t *count,
                      unsigned long long *stats, void *stream, const char *fn)
{
    SITING_REQUIRE(z != nullptr && count != nullptr, "%s: NULL terrain or output", fn);
    SITING_REQUIRE(nrows >= 2 && ncols >= 2, "%s: terrain must be at least 2x2", fn);
    SITING_REQUIRE(ld >= ncols, "%s: ld (%lld) < ncols (%lld)", fn, (long long)ld,
                   (long long)ncols);
    SITING_REQUIRE(roi >= 1 && roi <= kMaxRoi, "%s: roi %d outside 1..%d", fn, roi, kMaxRoi);
    SITING_REQUIRE(h_t >= 0 && h_t <= kMaxHeight && h_r >= 0 && h_r <= kMaxHeight,
                   "%s: heights outside 0..%d", fn, kMaxHeight);
    SITING_REQUIRE(K >= 1 && K <= 255, "%s: K %d outside 1..255", fn, K);
    if ((int64_t)(roi + 1) * ld >= ((int64_t)1 << 31)) {
        set_error("%s: roi*ld too large for 32-bit offsets", fn);
        return SITING_E_UNSUPPORTED;
    }
    // Largest tile side (multiple of 8, <= 128) whose haloed tile fits in LDS.
    int lds_max = device_max_lds();
    int T = 0;
    for (int c = 128; c >= 16; c -= 8) {
        int64_t bytes = (int64_t)(c + 2 * roi) * (c + 2 * roi) * 2;
        if (bytes <= lds_max) {
            T = c;
            break;
        }
    }
    bool use_lds = T > 0;
    if (!use_lds)
        T = 64;
    int64_t tiles_r = (nrows + T - 1) / T, tiles_c = (ncols + T - 1) / T;
    int64_t ntiles = tiles_r * tiles_c;
    int64_t per_xcd = (ntiles + 7) / 8;
    int64_t grid = per_xcd * 8;
    if (grid > INT32_MAX) {
        set_error("%s: terrain too large", fn);
        return SITING_E_UNSUPPORTED;
    }
    size_t lds = use_lds ? (size_t)(T + 2 * roi) * (T + 2 * roi) * 2 : 0;
    hipStream_t s = as_stream(stream);
    if (stats) {
        hipLaunchKernelGGL(vix_stats_reset, dim3(1), dim3(1), 0, s, stats);
        int rc = check_launch("vix_stats_reset");
        if (rc != SITING_OK)
            return rc;
    }
#define VIX_LAUNCH(LDS, CNT)                                                                    \
    hipLaunchKernelGGL((vix_kernel<LDS, CNT>), dim3((unsigned)grid), dim3(kVixThreads),        \
                       LDS ? lds : 0, s, z, nrows, ncols, ld, roi, h_t, h_r, K, seed, count, T, \
                       tiles_r, tiles_c, per_xcd, stats)
    if (use_lds && stats)
        VIX_LAUNCH(true, true);
    else if (use_lds)
        VIX_LAUNCH(true, false);
    else if (stats)
        VIX_LAUNCH(false, true);
    else
        VIX_LAUNCH(false, false);
#undef VIX_LAUNCH
    return check_launch("vix_kernel");
}

extern "C" int siting_vix(const int16_t *z, int64_t nrows, int64_t ncols, int64_t ld, int32_t roi,
                          int32_t h_t, int32_t h_r, int32_t K, uint64_t seed, uint8_t *count,
                          void *stream)
{
    clear_error();
    return vix_launch(z, nrows, ncols, ld, roi, h_t, h_r, K, seed, count, nullptr, stream,
                      "siting_vix");
}

extern "C" int siting_vix_stats(const int16_t *z, int64_t nrows, int64_t ncols, int64_t ld,
                                int32_t roi, int32_t h_t, int32_t h_r, int32_t K, uint64_t seed,
                                uint8_t *count, uint64_t *stats, void *stream)
{
    clear_error();
    SITING_REQUIRE(stats != nullptr, "siting_vix_stats: NULL stats");
    return vix_launch(z, nrows, ncols, ld, roi, h_t, h_r, K, seed, count,
                      reinterpret_cast<unsigned long long *>(stats), stream, "siting_vix_stats");
}
