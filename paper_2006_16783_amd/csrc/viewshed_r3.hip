// Exact per-cell viewsheds (the R3 family the paper cites as prior art for
// viewsheds): every lattice cell of an observer's ROI disk is tested by its
// own line of sight, the same test VIX runs (Definitions; "Terrain
// visibility": the segment sampled where it crosses grid lines of its major
// axis, the terrain linearly interpolated between the two adjacent posts,
// blocked only where the terrain is strictly above the segment).  O(R^3) per
// observer against the ray sweep's O(R^2): a measurement tool for how far the
// sweep's bitmaps are from exact line of sight, not part of the siting path.
//
// Design: persistent workgroups take observers round-robin; a wavefront
// takes one 64-bit word of the observer's window at a time, lane l testing
// column 64*word + l, so the word is a ballot and is written once, aligned
// to the global word grid like the sweep's bitmaps.  The terrain is read
// through the cache hierarchy; the comparisons are exact in int64.
#include <algorithm>

#include "common.hpp"

namespace siting {
namespace {

constexpr int kR3Waves = 4;

__device__ __forceinline__ bool los_clear(const int16_t *__restrict__ z, int64_t ld, int tx,
                                          int ty, int px, int py, int64_t E, int h_r)
{
    const int dx = px - tx, dy = py - ty;
    const int adx = dx < 0 ? -dx : dx, ady = dy < 0 ? -dy : dy;
    const bool xmajor = adx >= ady;
    const int n = xmajor ? adx : ady, mn = xmajor ? ady : adx;
    if (n <= 1)
        return true;
    // steps of the major and minor axes as element offsets
    const int64_t smaj = xmajor ? (dx < 0 ? -1 : 1) : (dy < 0 ? -ld : ld);
    const int64_t smin = xmajor ? (dy < 0 ? -ld : ld) : (dx < 0 ? -1 : 1);
    const int64_t Zt = (int64_t)z[(int64_t)py * ld + px] + h_r;
    const int64_t En = E * n, dZ = Zt - E;
    const int16_t *p = z + (int64_t)ty * ld + tx;
    int r = 0;
    for (int k = 1; k < n; k++) {
        // crossing k: minor offset q + r/n with k*mn = q*n + r
        p += smaj;
        r += mn;
        if (r >= n) {
            r -= n;
            p += smin;
        }
        const int64_t z0 = p[0];
        const int64_t z1 = r > 0 ? (int64_t)p[smin] : 0;
        const int64_t S = z0 * (n - r) + z1 * r;
        if (S > En + dZ * k)
            return false;
    }
    return true;
}

__global__ __launch_bounds__(64 * kR3Waves) void viewshed_r3_kernel(
    const int16_t *__restrict__ z, int64_t nrows, int64_t ncols, int64_t ld,
    const siting_observer *__restrict__ obs, int64_t n, const int64_t *__restrict__ offsets,
    uint64_t *__restrict__ bitmaps)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
        const siting_observer o = obs[i];
        if (o.roi < 1 || o.roi > kMaxRoi || o.x < 0 || o.x >= ncols || o.y < 0 ||
            o.y >= nrows || o.h_t < 0 || o.h_t > kMaxHeight || o.h_r < 0 ||
            o.h_r > kMaxHeight)
            continue;  // a record the host did not validate: its words stay untouched
        const int R = o.roi;
        const int64_t xlo = o.x - R < 0 ? 0 : o.x - R, xhi = o.x + R > ncols - 1 ? ncols - 1 : o.x + R;
        const int64_t ylo = o.y - R < 0 ? 0 : o.y - R, yhi = o.y + R > nrows - 1 ? nrows - 1 : o.y + R;
        const int64_t w0 = xlo >> 6;
        const int nw = (int)((xhi >> 6) - w0 + 1);
        const int rows = (int)(yhi - ylo + 1);
        const int64_t E = (int64_t)z[(int64_t)o.y * ld + o.x] + o.h_t;
        uint64_t *out = bitmaps + offsets[i];
        const int64_t R2 = (int64_t)R * R;
        for (int e = wave; e < rows * nw; e += kR3Waves) {
            const int row = e / nw, w = e - row * nw;
            const int64_t py = ylo + row, px = (w0 + w) * 64 + lane;
            const int64_t ddx = px - o.x, ddy = py - o.y;
            bool vis = false;
            if (px >= xlo && px <= xhi && ddx * ddx + ddy * ddy <= R2)
                vis = los_clear(z, ld, o.x, o.y, (int)px, (int)py, E, o.h_r);
            const uint64_t word = __ballot(vis);
            if (lane == 0)
                out[e] = word;
        }
    }
}

}  // namespace
}  // namespace siting

using namespace siting;

extern "C" int siting_viewshed_r3(const int16_t *z, int64_t nrows, int64_t ncols, int64_t ld,
                                  const siting_observer *obs, int64_t n, const int64_t *offsets,
                                  uint64_t *bitmaps, void *stream)
{
    clear_error();
    const char *fn = "siting_viewshed_r3";
    SITING_REQUIRE(n >= 0, "%s: n < 0", fn);
    SITING_REQUIRE(nrows >= 1 && ncols >= 1, "%s: empty terrain", fn);
    SITING_REQUIRE(ld >= ncols, "%s: ld < ncols", fn);
    if (n == 0)
        return SITING_OK;
    SITING_REQUIRE(z && obs && offsets && bitmaps, "%s: NULL device pointer", fn);
    if (ncols > INT32_MAX - 64 || nrows > INT32_MAX) {
        set_error("%s: terrain too large", fn);
        return SITING_E_UNSUPPORTED;
    }
    const int64_t grid = std::min<int64_t>(n, (int64_t)device_cus() * 8);
    hipLaunchKernelGGL(viewshed_r3_kernel, dim3((unsigned)grid), dim3(64 * kR3Waves), 0,
                       as_stream(stream), z, nrows, ncols, ld, obs, n, offsets, bitmaps);
    return check_launch("viewshed_r3_kernel");
}
