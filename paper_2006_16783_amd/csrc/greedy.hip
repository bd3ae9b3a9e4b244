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
//   bmax[b]  max of key[] over block b of 1024 candidates, with the round
//            stamp of that maximum (LDS)
// One persistent workgroup of 1024 threads runs every round.  The top key
// and the best key outside the top's block come from the block maxima.  The
// first pass of a round loads the top's window, its cumulative words and the
// keys of its block together (one window word and one key per thread); a
// stale top is re-evaluated, popcount(V & ~C), and taken at once if its exact
// key still exceeds every other key (the stated bound: gains only shrink), in
// which case its window is ORed into C from the words already loaded.  If it
// does not, later passes re-evaluate in parallel: the k-th involves the 2^k
// wavefronts with the best tops (at most 16), wavefront w owning the blocks
// b = w (mod 16).  The global top is always among them, so every pass makes
// progress; sparse candidate sets need one pass per round, dense ones (where
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

// popcount totals of a window: at most (2*16383+1)^2 < 2^31 bits
__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) { return wave_sum_u32((uint32_t)v); }

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
// wavefront (result in every lane); eight words per lane are loaded before
// any is used, so a window costs a few memory round trips
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
    for (int e0 = 0; e0 < words; e0 += 8 * 64) {
        uint64_t vv[8], cc[8];
#pragma unroll
        for (int u = 0; u < 8; u++) {
            const int e = e0 + u * 64 + lane;
            vv[u] = 0;
            cc[u] = 0;
            if (e < words) {
                const int row = e / w.nw, c = e - row * w.nw;
                vv[u] = v[e];
                cc[u] = C[(w.ylo + row) * W + w.w0 + c];
            }
        }
#pragma unroll
        for (int u = 0; u < 8; u++)
            cnt += __popcll(vv[u] & ~cc[u]);
    }
    return wave_sum_u64(cnt);
}

// max key of block b and that key's stamp, one wavefront (results in every
// lane); the key of candidate `ov` (if in the block) is taken as `ok` with
// stamp `of` instead of its stored value
__device__ __forceinline__ void wave_block_max(const uint64_t *key, const int32_t *fresh, int64_t n,
                                               int b, int lane, int64_t ov, uint64_t ok,
                                               int32_t of, uint64_t &best, int32_t &bfr)
{
    uint64_t v = 0;
    int32_t f = 0;
    const int64_t j0 = (int64_t)b * kGreedyBlock + lane;
    uint64_t kk[kGreedyBlock / 64];
    int32_t ff[kGreedyBlock / 64];
#pragma unroll
    for (int u = 0; u < kGreedyBlock / 64; u++) {
        const int64_t j = j0 + u * 64;
        kk[u] = 0;
        ff[u] = 0;
        if (j < n) {
            kk[u] = j == ov ? ok : key[j];
            ff[u] = j == ov ? of : fresh[j];
        }
    }
#pragma unroll
    for (int u = 0; u < kGreedyBlock / 64; u++) {
        if (kk[u] > v) {
            v = kk[u];
            f = ff[u];
        }
    }
    best = wave_max_u64(v);
    const uint64_t owner = __ballot(v == best && best != 0);
    bfr = __builtin_amdgcn_readlane(f, owner ? __ffsll((long long)owner) - 1 : 0);
}

__global__ __launch_bounds__(kGreedyThreads) void greedy_run(
    const uint64_t *__restrict__ bitmaps, const int64_t *__restrict__ offsets,
    const siting_observer *__restrict__ obs, int64_t n, int64_t nrows, int64_t ncols,
    int32_t max_obs, int64_t target, uint64_t *C, int64_t *__restrict__ selected,
    int64_t *__restrict__ gains, int32_t *__restrict__ nselected, uint64_t *key, int32_t *fresh)
{
    // block maxima of the keys and the round stamps of those maxima
    extern __shared__ uint64_t bmax[];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t W = (ncols + 63) >> 6;
    const int nblocks = (int)((n + kGreedyBlock - 1) / kGreedyBlock);
    int32_t *bfr = reinterpret_cast<int32_t *>(bmax + nblocks);
    // per-wavefront partials: s_t* for the top selection, s_a/s_b for the
    // pass's reduction (separate, so neither needs a barrier before reuse)
    __shared__ uint64_t s_t1[kGreedyWaves], s_t2[kGreedyWaves];
    __shared__ uint64_t s_a[kGreedyWaves], s_b[kGreedyWaves];

    // workgroup sum of a and max of b in one exchange (results in every
    // thread); s_a/s_b were last read before the previous round's final
    // barrier
    auto wg_sum_max = [&](uint64_t a, uint64_t b, uint64_t &sa, uint64_t &mb) {
        a = wave_sum_u64(a);
        b = wave_max_u64(b);
        if (lane == 0) {
            s_a[wave] = a;
            s_b[wave] = b;
        }
        __syncthreads();
        sa = 0;
        mb = 0;
        for (int w2 = 0; w2 < kGreedyWaves; w2++) {
            sa += s_a[w2];
            mb = s_b[w2] > mb ? s_b[w2] : mb;
        }
    };

    for (int b = wave; b < nblocks; b += kGreedyWaves) {
        uint64_t v;
        int32_t f;
        wave_block_max(key, fresh, n, b, lane, -1, 0, 0, v, f);
        if (lane == 0) {
            bmax[b] = v;
            bfr[b] = f;
        }
    }
    __syncthreads();

    int32_t t = 0;
    int64_t covered = 0;
    int pass = 0;
    while (t < max_obs && covered < target) {
        // ---- global top key and the best key outside its block
        uint64_t top = 0, second = 0, wmax = 0;
        int rank = 0;  // wavefronts holding a larger top than this one
        int wb = 0;    // this wavefront's best block
        if (pass == 0) {
            // every wavefront scans all block maxima itself: no exchange and
            // no barrier (the previous round's final barrier ordered the
            // block maxima it wrote)
            uint64_t m1 = 0, m2 = 0;
            for (int b = lane; b < nblocks; b += 64) {
                const uint64_t v = bmax[b];
                if (v > m1) {
                    m2 = m1;
                    m1 = v;
                } else if (v > m2) {
                    m2 = v;
                }
            }
            top = wave_max_u64(m1);
            const uint64_t owner = __ballot(m1 == top && top != 0);
            const int ol = owner ? __ffsll((long long)owner) - 1 : 0;
            second = wave_max_u64(lane == ol ? m2 : m1);
        } else {
            // stale passes rank the wavefronts' tops: every wavefront takes
            // the two largest of its blocks, then the workgroup
            uint64_t m1 = 0, m2 = 0;
            int b1 = -1;
            for (int b = wave + kGreedyWaves * lane; b < nblocks; b += kGreedyWaves * 64) {
                const uint64_t v = bmax[b];
                if (v > m1) {
                    m2 = m1;
                    m1 = v;
                    b1 = b;
                } else if (v > m2) {
                    m2 = v;
                }
            }
            wmax = wave_max_u64(m1);
            const uint64_t owner = __ballot(m1 == wmax && wmax != 0);
            const int ol = owner ? __ffsll((long long)owner) - 1 : 0;
            wb = __builtin_amdgcn_readlane(b1, ol);
            // the wavefront's second: the owner's own second or another lane's first
            const uint64_t wsec = wave_max_u64(lane == ol ? m2 : m1);
            if (lane == 0) {
                s_t1[wave] = wmax;
                s_t2[wave] = wsec;
            }
            __syncthreads();
            int tw = 0;
            for (int w2 = 0; w2 < kGreedyWaves; w2++) {
                const uint64_t v = s_t1[w2];
                if (v > top) {
                    top = v;
                    tw = w2;
                }
                rank += v > wmax;
            }
            for (int w2 = 0; w2 < kGreedyWaves; w2++) {
                const uint64_t v = w2 == tw ? s_t2[w2] : s_t1[w2];
                second = v > second ? v : second;
            }
        }
        const int64_t i = (int64_t)(0xFFFFFFFFull - (top & 0xFFFFFFFFull));
        const uint64_t g = top >> 32;
        if (top == 0 || i >= n)
            break;  // unreachable with n >= 1
        const int bi = (int)(i / kGreedyBlock);
        // (bmax/bfr change only after the pass's reduction barrier)
        const int32_t fr = bfr[bi];
        if (fr == t || pass == 0) {
            // Re-evaluate the top if it is stale (the whole workgroup, one
            // window word per thread), and take it if it is fresh or stays
            // above every other key.  The window, the cumulative words and the
            // top's block of keys are loaded together.
            const bool stale = fr != t;
            if (!stale && g == 0)
                break;
            const siting_observer o = obs[i];
            const bool valid = obs_ok(o, nrows, ncols);
            const int64_t j = (int64_t)bi * kGreedyBlock + tid;
            const uint64_t kj = j < n ? key[j] : 0;
            const int32_t fj = j < n ? fresh[j] : 0;
            Win w{0, 0, 0, 0};
            const uint64_t *v = bitmaps;
            if (valid) {
                w = window_of(o, nrows, ncols);
                v = bitmaps + offsets[i];
            }
            const int words = w.rows * w.nw;
            // this thread's first window word stays in registers for the OR
            uint64_t v0 = 0, c0 = 0;
            uint64_t cnt = 0;
            for (int e = tid; e < words; e += kGreedyThreads) {
                const int row = e / w.nw, c = e - row * w.nw;
                const uint64_t ve = v[e], ce = C[(w.ylo + row) * W + w.w0 + c];
                if (e == tid) {
                    v0 = ve;
                    c0 = ce;
                }
                cnt += __popcll(ve & ~ce);
            }
            // one exchange: the exact gain (when stale) and the largest key of
            // the top's block other than the top's own
            const uint64_t kj_ex = j == i ? 0 : kj;
            uint64_t gsum, bo;
            wg_sum_max(stale ? cnt : 0, kj_ex, gsum, bo);
            const uint64_t gain = stale ? gsum : g;
            const uint64_t nk = (gain << 32) | (0xFFFFFFFFull - (uint64_t)i);
            // lazy greedy: a fresh gain at least every other key (stale or
            // not) is the plain greedy choice; keys are unique
            const bool take = gain > 0 && (!stale || (nk > second && nk > bo));
            // after this pass: nk for i, or a zero gain once i is taken
            const uint64_t ki = take ? (0xFFFFFFFFull - (uint64_t)i) : nk;
            const int32_t fi = take ? t + 1 : t;
            const uint64_t bm2 = ki > bo ? ki : bo;
            // the holder of the block's new maximum records it (another
            // candidate's, or i's own new key)
            if ((bm2 == bo && kj_ex == bo && bo != 0) || (bm2 == ki && j == i)) {
                bmax[bi] = bm2;
                bfr[bi] = j == i ? fi : fj;
            }
            if (take) {
                for (int e = tid; e < words; e += kGreedyThreads) {
                    const int row = e / w.nw, c = e - row * w.nw;
                    uint64_t *ce = &C[(w.ylo + row) * W + w.w0 + c];
                    *ce = e == tid ? (c0 | v0) : (*ce | v[e]);
                }
            }
            if (j == i) {
                key[i] = ki;
                fresh[i] = fi;
            }
            if (tid == 0 && take) {
                selected[t] = i;
                gains[t] = (int64_t)gain;
            }
            if (take) {
                covered += (int64_t)gain;
                t++;
                pass = 0;
            } else {
                pass = 1;
            }
        } else {
            // later stale passes: the k-th re-evaluates the tops of the 2^k
            // best wavefronts in parallel, one wavefront each (up to 16)
            const bool go = wmax != 0 && rank < (1 << pass);
            pass = pass < 4 ? pass + 1 : 4;
            // ---- this wavefront re-evaluates the top of its best block
            const int64_t jj = (int64_t)(0xFFFFFFFFull - (wmax & 0xFFFFFFFFull));
            if (go && bfr[wb] != t) {
                const siting_observer o = obs[jj];
                uint64_t gj = 0;
                if (obs_ok(o, nrows, ncols))
                    gj = wave_gain(bitmaps, offsets, o, jj, nrows, ncols, C, W, lane);
                const uint64_t nkj = (gj << 32) | (0xFFFFFFFFull - (uint64_t)jj);
                uint64_t bv;
                int32_t bf;
                wave_block_max(key, fresh, n, wb, lane, jj, nkj, t, bv, bf);
                if (lane == 0) {
                    key[jj] = nkj;
                    fresh[jj] = t;
                    bmax[wb] = bv;
                    bfr[wb] = bf;
                }
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
        nblocks * 12 > kernel_max_dynamic_lds(reinterpret_cast<const void *>(&greedy_run))) {
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
    hipLaunchKernelGGL(greedy_run, dim3(1), dim3(kGreedyThreads), (size_t)nblocks * 12, s, bitmaps,
                       offsets, obs, n, nrows, ncols, max_obs, target_cells, cumulative, selected,
                       gains, nselected, key, fresh);
    return check_launch("greedy_run");
}
