// SITE: greedy selection of observers maximising the gain in cumulative
// viewshed area (stage Site; union by bitwise operations on 64-bit words),
// evaluated lazily with the stage's stated bound: a candidate's gain can only
// shrink as the cumulative viewshed grows, so a stale gain is an upper bound.
//
// State, all device-resident:
//   C        cumulative bitmap, nrows x ceil(ncols/64) uint64
//   key[i]   (gain bound << 32) | (2^32-1 - i): one 64-bit max gives the
//            largest bound with ties to the smallest index
//   fresh[i] the round in which key[i] was last computed exactly
//   bmax[b]  max of key[] over block b of 1024 candidates (LDS)
// One persistent workgroup of 1024 threads runs every round.  If the global
// top key is fresh it is exactly the plain greedy argmax and is taken (its
// window ORed into C).  Otherwise wavefronts re-evaluate in parallel:
// wavefront w owns the blocks b = w (mod 16) and recomputes the top
// candidate of its best block, popcount(V & ~C) over the window, then that
// block's maximum.  The first stale pass of a round re-evaluates only the
// global top, with the whole workgroup (one window word per thread); the
// k-th later pass involves the 2^k wavefronts with the best tops (at most
// 16).  The global top is always among them, so every pass makes progress;
// sparse candidate sets need one re-evaluation per round, dense ones (where
// a selection leaves many stale neighbours on top) converge in a few wide
// passes.
#include <algorithm>

#include "common.hpp"

namespace siting {
namespace {

constexpr int kGreedyThreads = 1024;
constexpr int kGreedyWaves = kGreedyThreads / 64;
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
    const siting_observer o = obs[i];
    if (lane == 0)
        fresh[i] = 0;
    if (!obs_ok(o, nrows, ncols)) {  // an invalid record never gains
        if (lane == 0)
            key[i] = 0xFFFFFFFFull - (uint64_t)i;
        return;
    }
    const uint64_t *v = bitmaps + offsets[i];
    int64_t words = offsets[i + 1] - offsets[i];
    uint64_t g = 0;
    for (int64_t e = lane; e < words; e += 64)
        g += __popcll(v[e]);
    g = wave_sum_u64(g);
    if (lane == 0)
        key[i] = (g << 32) | (0xFFFFFFFFull - (uint64_t)i);
}

// gain of candidate j against C: popcount(V_j & ~C) over its window, one
// wavefront (result in every lane)
__device__ __forceinline__ uint64_t wave_gain(const uint64_t *__restrict__ bitmaps,
                                              const int64_t *__restrict__ offsets,
                                              const siting_observer &o, int64_t j, int64_t nrows,
                                              int64_t ncols, const uint64_t *C, int64_t W,
                                              int lane)
{
    const Win w = window_of(o, nrows, ncols);
    const uint64_t *v = bitmaps + offsets[j];
    const int words = w.rows * w.nw;
    uint64_t cnt = 0;
    for (int e = lane; e < words; e += 64) {
        const int row = e / w.nw, c = e - row * w.nw;
        cnt += __popcll(v[e] & ~C[(w.ylo + row) * W + w.w0 + c]);
    }
    return wave_sum_u64(cnt);
}

// max key of block b, one wavefront (result in every lane)
__device__ __forceinline__ uint64_t wave_block_max(const uint64_t *key, int64_t n, int b, int lane)
{
    uint64_t v = 0;
    for (int64_t j = (int64_t)b * kGreedyBlock + lane; j < n && j < (int64_t)(b + 1) * kGreedyBlock;
         j += 64)
        v = key[j] > v ? key[j] : v;
    return wave_max_u64(v);
}

__global__ __launch_bounds__(kGreedyThreads) void greedy_run(
    const uint64_t *__restrict__ bitmaps, const int64_t *__restrict__ offsets,
    const siting_observer *__restrict__ obs, int64_t n, int64_t nrows, int64_t ncols,
    int32_t max_obs, int64_t target, uint64_t *C, int64_t *__restrict__ selected,
    int64_t *__restrict__ gains, int32_t *__restrict__ nselected, uint64_t *key, int32_t *fresh)
{
    extern __shared__ uint64_t bmax[];
    __shared__ uint64_t s_red[kGreedyWaves];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t W = (ncols + 63) >> 6;
    const int nblocks = (int)((n + kGreedyBlock - 1) / kGreedyBlock);

    // workgroup-wide reductions (result in every thread)
    auto wg_reduce = [&](uint64_t v, bool is_max) -> uint64_t {
        v = is_max ? wave_max_u64(v) : wave_sum_u64(v);
        __syncthreads();
        if (lane == 0)
            s_red[wave] = v;
        __syncthreads();
        uint64_t r = is_max ? 0 : 0;
        for (int w2 = 0; w2 < kGreedyWaves; w2++)
            r = is_max ? (s_red[w2] > r ? s_red[w2] : r) : r + s_red[w2];
        __syncthreads();
        return r;
    };
    // workgroup-wide refresh of bmax[b] (one key per thread)
    auto wg_refresh = [&](int b) {
        const int64_t j = (int64_t)b * kGreedyBlock + tid;
        const uint64_t v = wg_reduce(j < n ? key[j] : 0, true);
        if (tid == 0)
            bmax[b] = v;
    };

    for (int b = wave; b < nblocks; b += kGreedyWaves) {
        const uint64_t v = wave_block_max(key, n, b, lane);
        if (lane == 0)
            bmax[b] = v;
    }
    __syncthreads();

    int32_t t = 0;
    int64_t covered = 0;
    int pass = 0;
    while (t < max_obs && covered < target) {
        // ---- global top key: every wavefront takes the max over its blocks
        // (kept for the re-evaluation below), then the workgroup max
        uint64_t mine = 0;
        int myb = -1;
        // lanes stride over this wavefront's blocks
        for (int b = wave + kGreedyWaves * lane; b < nblocks; b += kGreedyWaves * 64) {
            const uint64_t v = bmax[b];
            if (v > mine) {
                mine = v;
                myb = b;
            }
        }
        // wavefront argmax (keys are unique, so the owner lane is unique)
        const uint64_t wmax = wave_max_u64(mine);
        const uint64_t owner = __ballot(mine == wmax && wmax != 0);
        const int wb = __shfl(myb, owner ? __ffsll((long long)owner) - 1 : 0, 64);
        if (lane == 0)
            s_red[wave] = wmax;
        __syncthreads();
        uint64_t top = 0;
        int rank = 0;  // wavefronts holding a larger top than this one
        for (int w2 = 0; w2 < kGreedyWaves; w2++) {
            const uint64_t v = s_red[w2];
            top = v > top ? v : top;
            rank += v > wmax;
        }
        const int64_t i = (int64_t)(0xFFFFFFFFull - (top & 0xFFFFFFFFull));
        const uint64_t g = top >> 32;
        if (top == 0 || i >= n)
            break;  // unreachable with n >= 1
        const int32_t fr = fresh[i];
        __syncthreads();  // every thread has read s_red and fresh[i]
        if (fr == t) {
            if (g == 0)
                break;
            const Win w = window_of(obs[i], nrows, ncols);
            const uint64_t *v = bitmaps + offsets[i];
            for (int e = tid; e < w.rows * w.nw; e += kGreedyThreads) {
                const int row = e / w.nw, c = e - row * w.nw;
                C[(w.ylo + row) * W + w.w0 + c] |= v[e];
            }
            if (tid == 0) {
                selected[t] = i;
                gains[t] = (int64_t)g;
                key[i] = 0xFFFFFFFFull - (uint64_t)i;  // gains nothing from now on
                fresh[i] = t + 1;
            }
            __syncthreads();
            wg_refresh((int)(i / kGreedyBlock));
            covered += (int64_t)g;
            t++;
            pass = 0;
        } else if (pass == 0) {
            // first stale pass of a round: the whole workgroup re-evaluates
            // the global top (one word per thread), then refreshes its block
            const siting_observer o = obs[i];
            uint64_t cnt = 0;
            if (obs_ok(o, nrows, ncols)) {
                const Win w = window_of(o, nrows, ncols);
                const uint64_t *v = bitmaps + offsets[i];
                for (int e = tid; e < w.rows * w.nw; e += kGreedyThreads) {
                    const int row = e / w.nw, c = e - row * w.nw;
                    cnt += __popcll(v[e] & ~C[(w.ylo + row) * W + w.w0 + c]);
                }
            }
            cnt = wg_reduce(cnt, false);
            if (tid == 0) {
                key[i] = (cnt << 32) | (0xFFFFFFFFull - (uint64_t)i);
                fresh[i] = t;
            }
            __syncthreads();
            wg_refresh((int)(i / kGreedyBlock));
            pass = 1;
        } else {
            // later stale passes: the k-th re-evaluates the tops of the 2^k
            // best wavefronts in parallel, one wavefront each (up to 16)
            const bool go = wmax != 0 && rank < (1 << pass);
            pass = pass < 4 ? pass + 1 : 4;
            // ---- this wavefront re-evaluates the top of its best block
            const int64_t j = (int64_t)(0xFFFFFFFFull - (wmax & 0xFFFFFFFFull));
            if (go && fresh[j] != t) {
                const siting_observer o = obs[j];
                uint64_t gj = 0;
                if (obs_ok(o, nrows, ncols))
                    gj = wave_gain(bitmaps, offsets, o, j, nrows, ncols, C, W, lane);
                if (lane == 0) {
                    key[j] = (gj << 32) | (0xFFFFFFFFull - (uint64_t)j);
                    fresh[j] = t;
                }
                const uint64_t bv = wave_block_max(key, n, wb, lane);
                if (lane == 0)
                    bmax[wb] = bv;
            }
        }
        __syncthreads();
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
    const size_t need = siting_greedy_workspace_size(n);
    if (ws == nullptr || ws_bytes < need) {
        set_error("%s: workspace of %zu bytes needed", fn, need);
        return SITING_E_WORKSPACE;
    }
    const int64_t nblocks = (n + kGreedyBlock - 1) / kGreedyBlock;
    if (nblocks > kGreedyMaxBlocks ||
        nblocks * 8 > kernel_max_dynamic_lds(reinterpret_cast<const void *>(&greedy_run))) {
        set_error("%s: %lld candidates exceed the supported maximum", fn, (long long)n);
        return SITING_E_UNSUPPORTED;
    }
    uint64_t *key = reinterpret_cast<uint64_t *>(ws);
    int32_t *fresh =
        reinterpret_cast<int32_t *>(reinterpret_cast<char *>(ws) + align256((size_t)n * 8));
    hipStream_t s = as_stream(stream);
    const int64_t W = (ncols + 63) / 64;
    const int64_t cwords = nrows * W;
    const int zg = (int)std::min<int64_t>((cwords + 255) / 256, (int64_t)device_cus() * 16);
    int rc;
    hipLaunchKernelGGL(greedy_zero, dim3(zg > 0 ? zg : 1), dim3(256), 0, s, cumulative, cwords);
    if ((rc = check_launch("greedy_zero")) != SITING_OK)
        return rc;
    hipLaunchKernelGGL(greedy_init, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, bitmaps,
                       offsets, obs, n, nrows, ncols, key, fresh);
    if ((rc = check_launch("greedy_init")) != SITING_OK)
        return rc;
    hipLaunchKernelGGL(greedy_run, dim3(1), dim3(kGreedyThreads), (size_t)nblocks * 8, s, bitmaps,
                       offsets, obs, n, nrows, ncols, max_obs, target_cells, cumulative, selected,
                       gains, nselected, key, fresh);
    return check_launch("greedy_run");
}
