// SITE: greedy selection of observers maximising the gain in cumulative
// viewshed area (stage Site; union by bitwise operations on 64-bit words),
// evaluated lazily with the stage's stated bound: a candidate's gain can only
// shrink as the cumulative viewshed grows.
//
// State, all device-resident:
//   C        cumulative bitmap, nrows x ceil(ncols/64) uint64
//   key[i]   (gain bound << 32) | (2^32-1 - i): one 64-bit max gives the
//            largest bound with ties to the smallest index
//   fresh[i] the round in which key[i] was last computed exactly
//   bmax[b]  max of key[] over block b of 1024 candidates (LDS)
// One persistent workgroup of 1024 threads runs every round: argmax over
// bmax, then either accept the top candidate (fresh) and OR its window into
// C, or recompute its exact gain popcount(V & ~C) over its window and
// refresh its block maximum.  Taking the top only when fresh makes the
// choice exactly the plain greedy argmax.
#include "common.hpp"

namespace siting {
namespace {

constexpr int kGreedyThreads = 1024;
constexpr int kGreedyBlock = 1024;   // candidates per bmax entry
constexpr int kGreedyMaxBlocks = 16384;

__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        uint64_t w = __shfl_xor(v, o, 64);
        v = w > v ? w : v;
    }
    return v;
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1)
        v += __shfl_xor(v, o, 64);
    return v;
}

struct Win {
    int64_t ylo, w0;
    int rows, nw;
};

__device__ __forceinline__ Win window_of(const siting_observer &o, int64_t nrows, int64_t ncols)
{
    Win w;
    int64_t R = o.roi;
    int64_t xlo = o.x - R < 0 ? 0 : o.x - R, xhi = o.x + R > ncols - 1 ? ncols - 1 : o.x + R;
    w.ylo = o.y - R < 0 ? 0 : o.y - R;
    int64_t yhi = o.y + R > nrows - 1 ? nrows - 1 : o.y + R;
    w.w0 = xlo >> 6;
    w.nw = (int)((xhi >> 6) - w.w0 + 1);
    w.rows = (int)(yhi - w.ylo + 1);
    return w;
}

__global__ void greedy_zero(uint64_t *__restrict__ c, int64_t words)
{
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < words; e += stride)
        c[e] = 0;
}

// Initial keys: gain against the empty cumulative viewshed = popcount(V_i);
// one wavefront per candidate.
__device__ __forceinline__ bool obs_ok(const siting_observer &o, int64_t nrows, int64_t ncols)
{
    return o.roi >= 1 && o.roi <= kMaxRoi && o.x >= 0 && o.x < ncols && o.y >= 0 && o.y < nrows;
}

__global__ __launch_bounds__(256) void greedy_init(const uint64_t *__restrict__ bitmaps,
                                                   const int64_t *__restrict__ offsets,
                                                   const siting_observer *__restrict__ obs,
                                                   int64_t n, int64_t nrows, int64_t ncols,
                                                   uint64_t *__restrict__ key,
                                                   int32_t *__restrict__ fresh)
{
    int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    int lane = threadIdx.x & 63;
    if (i >= n)
        return;
    if (!obs_ok(obs[i], nrows, ncols)) {  // an invalid record never gains
        if (lane == 0) {
            key[i] = 0xFFFFFFFFull - (uint64_t)i;
            fresh[i] = 0;
        }
        return;
    }
    const uint64_t *v = bitmaps + offsets[i];
    int64_t words = offsets[i + 1] - offsets[i];
    uint64_t g = 0;
    for (int64_t e = lane; e < words; e += 64)
        g += __popcll(v[e]);
    g = wave_sum_u64(g);
    if (lane == 0) {
        key[i] = (g << 32) | (0xFFFFFFFFull - (uint64_t)i);
        fresh[i] = 0;
    }
}

__global__ __launch_bounds__(kGreedyThreads) void greedy_lazy(
    const uint64_t *__restrict__ bitmaps, const int64_t *__restrict__ offsets,
    const siting_observer *__restrict__ obs, int64_t n, int64_t nrows, int64_t ncols,
    int32_t max_obs, int64_t target, uint64_t *C, int64_t *__restrict__ selected,
    int64_t *__restrict__ gains, int32_t *__restrict__ nselected, uint64_t *key, int32_t *fresh)
{
    extern __shared__ uint64_t bmax[];
    __shared__ uint64_t s_red[kGreedyThreads / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nwaves = kGreedyThreads / 64;
    const int64_t W = (ncols + 63) >> 6;
    const int nblocks = (int)((n + kGreedyBlock - 1) / kGreedyBlock);

    // block-wide reductions (result valid in every thread)
    auto block_max = [&](uint64_t v) -> uint64_t {
        v = wave_max_u64(v);
        if (lane == 0)
            s_red[wave] = v;
        __syncthreads();
        uint64_t r = s_red[0];
        for (int w = 1; w < nwaves; w++)
            r = s_red[w] > r ? s_red[w] : r;
        __syncthreads();
        return r;
    };
    auto block_sum = [&](uint64_t v) -> uint64_t {
        v = wave_sum_u64(v);
        if (lane == 0)
            s_red[wave] = v;
        __syncthreads();
        uint64_t r = 0;
        for (int w = 0; w < nwaves; w++)
            r += s_red[w];
        __syncthreads();
        return r;
    };
    auto refresh_block = [&](int b) {
        int64_t j = (int64_t)b * kGreedyBlock + tid;
        uint64_t v = j < n ? key[j] : 0;
        v = block_max(v);
        if (tid == 0)
            bmax[b] = v;
        __syncthreads();
    };

    for (int b = wave; b < nblocks; b += nwaves) {
        uint64_t v = 0;
        for (int64_t j = (int64_t)b * kGreedyBlock + lane; j < n && j < (int64_t)(b + 1) * kGreedyBlock; j += 64)
            v = key[j] > v ? key[j] : v;
        v = wave_max_u64(v);
        if (lane == 0)
            bmax[b] = v;
    }
    __syncthreads();

    int32_t t = 0;
    int64_t covered = 0;
    while (t < max_obs && covered < target) {
        uint64_t top = 0;
        for (int b = tid; b < nblocks; b += kGreedyThreads)
            top = bmax[b] > top ? bmax[b] : top;
        top = block_max(top);
        int64_t i = (int64_t)(0xFFFFFFFFull - (top & 0xFFFFFFFFull));
        uint64_t g = top >> 32;
        if (i >= n)
            break;  // unreachable with n >= 1
        const siting_observer o = obs[i];
        if (!obs_ok(o, nrows, ncols)) {
            // never selected: its gain is 0 from the start
            if (g == 0)
                break;
            __syncthreads();
            if (tid == 0) {
                key[i] = 0xFFFFFFFFull - (uint64_t)i;
                fresh[i] = t;
            }
            __syncthreads();
            refresh_block((int)(i / kGreedyBlock));
            continue;
        }
        const Win w = window_of(o, nrows, ncols);
        const uint64_t *v = bitmaps + offsets[i];
        const int words = w.rows * w.nw;
        const int32_t fr = fresh[i];
        __syncthreads();  // every thread has read fresh[i] before it changes
        if (fr == t) {
            if (g == 0)
                break;
            for (int e = tid; e < words; e += kGreedyThreads) {
                int row = e / w.nw, c = e - row * w.nw;
                uint64_t *cw = C + (w.ylo + row) * W + w.w0 + c;
                *cw |= v[e];
            }
            if (tid == 0) {
                selected[t] = i;
                gains[t] = (int64_t)g;
                key[i] = 0xFFFFFFFFull - (uint64_t)i;  // gain 0 from now on
                fresh[i] = t + 1;
            }
            covered += (int64_t)g;
            t++;
        } else {
            uint64_t cnt = 0;
            for (int e = tid; e < words; e += kGreedyThreads) {
                int row = e / w.nw, c = e - row * w.nw;
                cnt += __popcll(v[e] & ~C[(w.ylo + row) * W + w.w0 + c]);
            }
            cnt = block_sum(cnt);
            if (tid == 0) {
                key[i] = (cnt << 32) | (0xFFFFFFFFull - (uint64_t)i);
                fresh[i] = t;
            }
        }
        __syncthreads();
        refresh_block((int)(i / kGreedyBlock));
    }
    if (tid == 0)
        *nselected = t;
}

}  // namespace
}  // namespace siting

using namespace siting;

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

extern "C" size_t siting_greedy_workspace_size(int64_t n)
{
    if (n < 0)
        return 0;
    return align256((size_t)n * 8) + align256((size_t)n * 4);
}

extern "C" int siting_greedy(const uint64_t *bitmaps, const int64_t *offsets,
                             const siting_observer *obs, int64_t n, int64_t nrows, int64_t ncols,
                             int32_t max_obs, int64_t target_cells, uint64_t *cumulative,
                             int64_t *selected, int64_t *gains, int32_t *nselected, void *ws,
                             size_t ws_bytes, void *stream)
{
    clear_error();
    const char *fn = "siting_greedy";
    SITING_REQUIRE(n >= 1 && n < 0xFFFFFFFFll, "%s: n must be in 1..2^32-2", fn);
    SITING_REQUIRE(nrows >= 1 && ncols >= 1, "%s: empty terrain", fn);
    SITING_REQUIRE(max_obs >= 0, "%s: max_obs < 0", fn);
    SITING_REQUIRE(bitmaps && offsets && obs && cumulative && nselected,
                   "%s: NULL device pointer", fn);
    SITING_REQUIRE(max_obs == 0 || (selected && gains), "%s: NULL selected/gains", fn);
    if (ws == nullptr || ws_bytes < siting_greedy_workspace_size(n)) {
        set_error("%s: workspace of %zu bytes needed", fn, siting_greedy_workspace_size(n));
        return SITING_E_WORKSPACE;
    }
    int64_t nblocks = (n + kGreedyBlock - 1) / kGreedyBlock;
    if (nblocks > kGreedyMaxBlocks || nblocks * 8 > device_max_lds()) {
        set_error("%s: %lld candidates exceed the supported maximum", fn, (long long)n);
        return SITING_E_UNSUPPORTED;
    }
    uint64_t *key = reinterpret_cast<uint64_t *>(ws);
    int32_t *fresh = reinterpret_cast<int32_t *>(reinterpret_cast<char *>(ws) + align256((size_t)n * 8));
    hipStream_t s = as_stream(stream);
    int64_t W = (ncols + 63) / 64;
    int64_t cwords = nrows * W;
    int zg = (int)std::min<int64_t>((cwords + 255) / 256, (int64_t)device_cus() * 16);
    hipLaunchKernelGGL(greedy_zero, dim3(zg > 0 ? zg : 1), dim3(256), 0, s, cumulative, cwords);
    int rc = check_launch("greedy_zero");
    if (rc != SITING_OK)
        return rc;
    hipLaunchKernelGGL(greedy_init, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, bitmaps,
                       offsets, obs, n, nrows, ncols, key, fresh);
    rc = check_launch("greedy_init");
    if (rc != SITING_OK)
        return rc;
    hipLaunchKernelGGL(greedy_lazy, dim3(1), dim3(kGreedyThreads), (size_t)nblocks * 8, s, bitmaps,
                       offsets, obs, n, nrows, ncols, max_obs, target_cells, cumulative, selected,
                       gains, nselected, key, fresh);
    return check_launch("greedy_lazy");
}
