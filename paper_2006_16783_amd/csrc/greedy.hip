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
//   bmax[b]  max of key[] over block b of 512 candidates, with the round
//            stamp of that maximum (LDS)
// One wavefront runs every round, so a round needs no barrier: the top key
// and the best key outside the top's block come from the block maxima; the
// top's window words, its cumulative words and the keys of its block are then
// loaded together (16 window words and 8 keys per lane); a stale top is
// re-evaluated, popcount(V & ~C), and taken at once if its exact key still
// exceeds every other key (the stated bound: gains only shrink), its window
// ORed into C from the words already in registers.  Otherwise its new key goes
// back and the next round pops the new top: each round either selects an
// observer or lowers a key, and a fresh top (re-evaluated since the last
// selection) is exact and taken without loading its gain again.
#include <algorithm>

#include "common.hpp"

namespace siting {
namespace {

constexpr int kGreedyBlock = 512;    // candidates per bmax entry
constexpr int kGreedyKeys = kGreedyBlock / 64;  // keys of a block per lane
constexpr int kGreedyWords = 16;     // window words per lane per batch
constexpr int kGreedyMaxBlocks = 8192;

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

// block maxima of the initial keys, one wavefront per block
__global__ __launch_bounds__(64) void greedy_blocks(const uint64_t *__restrict__ key,
                                                    const int32_t *__restrict__ fresh, int64_t n,
                                                    uint64_t *__restrict__ bmax_g,
                                                    int32_t *__restrict__ bfr_g)
{
    const int b = blockIdx.x, lane = threadIdx.x;
    uint64_t v;
    int32_t f;
    wave_block_max(key, fresh, n, b, lane, -1, 0, 0, v, f);
    if (lane == 0) {
        bmax_g[b] = v;
        bfr_g[b] = f;
    }
}

__global__ __launch_bounds__(64) void greedy_run(
    const uint64_t *__restrict__ bitmaps, const int64_t *__restrict__ offsets,
    const siting_observer *__restrict__ obs, int64_t n, int64_t nrows, int64_t ncols,
    int32_t max_obs, int64_t target, uint64_t *C, int64_t *__restrict__ selected,
    int64_t *__restrict__ gains, int32_t *__restrict__ nselected, uint64_t *key, int32_t *fresh,
    const uint64_t *__restrict__ bmax_g, const int32_t *__restrict__ bfr_g)
{
    // block maxima of the keys and the round stamps of those maxima
    extern __shared__ uint64_t bmax[];
    const int lane = threadIdx.x;
    const int64_t W = (ncols + 63) >> 6;
    const int nblocks = (int)((n + kGreedyBlock - 1) / kGreedyBlock);
    int32_t *bfr = reinterpret_cast<int32_t *>(bmax + nblocks);
    for (int b = lane; b < nblocks; b += 64) {
        bmax[b] = bmax_g[b];
        bfr[b] = bfr_g[b];
    }
    // one wavefront: LDS accesses run in order; the barrier only keeps the
    // compiler from moving them
    __syncthreads();

    int32_t t = 0;
    int64_t covered = 0;
    // the next round's top is known when a round ends (the larger of the best
    // key outside the round's block and that block's new maximum): its record
    // and its block's keys are loaded then, while the next top selection runs
    int64_t pf_i = -1;
    siting_observer pf_o{0, 0, 0, 0, 0};
    int64_t pf_off = 0;
    uint64_t pf_k[kGreedyKeys];
    int32_t pf_f[kGreedyKeys];
    auto load_block = [&](int b, int64_t skip, uint64_t *kk, int32_t *ff) {
#pragma unroll
        for (int u = 0; u < kGreedyKeys; u++) {
            const int64_t j = (int64_t)b * kGreedyBlock + u * 64 + lane;
            kk[u] = j < n && j != skip ? key[j] : 0;
            ff[u] = j < n ? fresh[j] : 0;
        }
    };
    while (t < max_obs && covered < target) {
        // ---- the top key and the best key outside its block
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
        const uint64_t top = wave_max_u64(m1);
        const uint64_t owner = __ballot(m1 == top && top != 0);
        const int ol = owner ? __ffsll((long long)owner) - 1 : 0;
        const uint64_t second = wave_max_u64(lane == ol ? m2 : m1);
        const int64_t i = (int64_t)(0xFFFFFFFFull - (top & 0xFFFFFFFFull));
        const uint64_t g = top >> 32;
        if (top == 0 || i >= n)
            break;  // unreachable with n >= 1
        const int bi = (int)(i / kGreedyBlock);
        const int32_t fr = bfr[bi];
        const bool stale = fr != t;
        if (!stale && g == 0)
            break;  // no candidate gains anything
        // ---- the top's window, its cumulative words and its block's keys,
        // loaded together
        siting_observer o;
        int64_t off;
        uint64_t kk[kGreedyKeys];
        int32_t ff[kGreedyKeys];
        if (i == pf_i) {
            o = pf_o;
            off = pf_off;
#pragma unroll
            for (int u = 0; u < kGreedyKeys; u++) {
                kk[u] = pf_k[u];
                ff[u] = pf_f[u];
            }
        } else {
            o = obs[i];
            off = offsets[i];
            load_block(bi, i, kk, ff);
        }
        const bool valid = obs_ok(o, nrows, ncols);
        Win w{0, 0, 0, 0};
        const uint64_t *v = bitmaps;
        if (valid) {
            w = window_of(o, nrows, ncols);
            v = bitmaps + off;
        }
        const int words = w.rows * w.nw;
        // the first batch of window words stays in registers for the OR; the
        // word index e = 64u + lane walks the window's rows without division
        const int dq = 64 / (w.nw > 0 ? w.nw : 1), dr = 64 - dq * w.nw;
        int row0 = lane / (w.nw > 0 ? w.nw : 1), col0 = lane - row0 * w.nw;
        int64_t cix[kGreedyWords];
        uint64_t vv[kGreedyWords], cc[kGreedyWords];
        {
            int row = row0, col = col0;
#pragma unroll
            for (int u = 0; u < kGreedyWords; u++) {
                cix[u] = (w.ylo + row) * W + w.w0 + col;
                col += dr;
                row += dq;
                if (col >= w.nw) {
                    col -= w.nw;
                    row++;
                }
            }
        }
#pragma unroll
        for (int u = 0; u < kGreedyWords; u++) {
            const int e = u * 64 + lane;
            vv[u] = 0;
            cc[u] = 0;
            if (e < words) {
                vv[u] = v[e];
                cc[u] = C[cix[u]];
            }
        }
        uint64_t cnt = 0;
#pragma unroll
        for (int u = 0; u < kGreedyWords; u++)
            cnt += __popcll(vv[u] & ~cc[u]);
        // windows above 64 * kGreedyWords words: the rest in further batches
        for (int e0 = 64 * kGreedyWords; stale && e0 < words; e0 += 64 * kGreedyWords) {
            uint64_t v2[kGreedyWords], c2[kGreedyWords];
#pragma unroll
            for (int u = 0; u < kGreedyWords; u++) {
                const int e = e0 + u * 64 + lane;
                v2[u] = 0;
                c2[u] = 0;
                if (e < words) {
                    const int row = e / w.nw, c = e - row * w.nw;
                    v2[u] = v[e];
                    c2[u] = C[(w.ylo + row) * W + w.w0 + c];
                }
            }
#pragma unroll
            for (int u = 0; u < kGreedyWords; u++)
                cnt += __popcll(v2[u] & ~c2[u]);
        }
        // the largest key of the top's block other than the top's own
        uint64_t kb = 0;
        int32_t fb = 0;
#pragma unroll
        for (int u = 0; u < kGreedyKeys; u++) {
            if (kk[u] > kb) {
                kb = kk[u];
                fb = ff[u];
            }
        }
        const uint64_t bo = wave_max_u64(kb);
        const uint64_t bown = __ballot(kb == bo && bo != 0);
        const int32_t fbo = __builtin_amdgcn_readlane(fb, bown ? __ffsll((long long)bown) - 1 : 0);
        const uint64_t gain = stale ? wave_sum_u64(cnt) : g;
        const uint64_t nk = (gain << 32) | (0xFFFFFFFFull - (uint64_t)i);
        // lazy greedy: a fresh gain at least every other key (stale or not)
        // is the plain greedy choice; keys are unique
        const bool take = gain > 0 && (!stale || (nk > second && nk > bo));
        // after this round: nk for i, or a zero gain once i is taken
        const uint64_t ki = take ? (0xFFFFFFFFull - (uint64_t)i) : nk;
        const int32_t fi = take ? t + 1 : t;
        if (lane == 0) {
            const bool mine = ki > bo;
            bmax[bi] = mine ? ki : bo;
            bfr[bi] = mine ? fi : fbo;
            key[i] = ki;
            fresh[i] = fi;
            if (take) {
                selected[t] = i;
                gains[t] = (int64_t)gain;
            }
        }
        if (take) {
#pragma unroll
            for (int u = 0; u < kGreedyWords; u++) {
                const int e = u * 64 + lane;
                if (e < words)
                    C[cix[u]] = cc[u] | vv[u];
            }
            for (int e = 64 * kGreedyWords + lane; e < words; e += 64) {
                const int row = e / w.nw, c = e - row * w.nw;
                uint64_t *ce = &C[(w.ylo + row) * W + w.w0 + c];
                *ce |= v[e];
            }
            covered += (int64_t)gain;
            t++;
        }
        // the next top: the best key outside block bi or bi's new maximum
        {
            const uint64_t bnew = ki > bo ? ki : bo;
            const uint64_t nx = second > bnew ? second : bnew;
            const int64_t p = (int64_t)(0xFFFFFFFFull - (nx & 0xFFFFFFFFull));
            pf_i = nx != 0 && p < n ? p : -1;
            if (pf_i >= 0) {
                pf_o = obs[pf_i];
                pf_off = offsets[pf_i];
                // keys of the next top's block; i's key and stamp as just set
                load_block((int)(pf_i / kGreedyBlock), pf_i, pf_k, pf_f);
#pragma unroll
                for (int u = 0; u < kGreedyKeys; u++) {
                    const int64_t j = (pf_i / kGreedyBlock) * kGreedyBlock + u * 64 + lane;
                    if (j == i && j != pf_i) {  // the top's own key stays out
                        pf_k[u] = ki;
                        pf_f[u] = fi;
                    }
                }
            }
        }
        __syncthreads();
    }
    if (lane == 0)
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
    const size_t nb = (size_t)((n + kGreedyBlock - 1) / kGreedyBlock);
    return align256((size_t)n * 8) + align256((size_t)n * 4) + align256(nb * 8) + align256(nb * 4);
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
    char *wsb = reinterpret_cast<char *>(ws);
    uint64_t *key = reinterpret_cast<uint64_t *>(wsb);
    wsb += align256((size_t)n * 8);
    int32_t *fresh = reinterpret_cast<int32_t *>(wsb);
    wsb += align256((size_t)n * 4);
    uint64_t *bmax_g = reinterpret_cast<uint64_t *>(wsb);
    wsb += align256((size_t)nblocks * 8);
    int32_t *bfr_g = reinterpret_cast<int32_t *>(wsb);
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
    hipLaunchKernelGGL(greedy_blocks, dim3((unsigned)nblocks), dim3(64), 0, s, key, fresh, n,
                       bmax_g, bfr_g);
    if ((rc = check_launch("greedy_blocks")) != SITING_OK)
        return rc;
    hipLaunchKernelGGL(greedy_run, dim3(1), dim3(64), (size_t)nblocks * 12, s, bitmaps, offsets,
                       obs, n, nrows, ncols, max_obs, target_cells, cumulative, selected, gains,
                       nselected, key, fresh, bmax_g, bfr_g);
    return check_launch("greedy_run");
}
