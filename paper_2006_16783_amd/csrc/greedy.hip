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
//
// Windows above one batch (1024 words: ROI above about 125) make a round
// latency-bound on one wavefront's loads, so when the largest window exceeds a
// batch a second instantiation runs instead: wavefront 0 still runs every
// round alone, and three more wavefronts, waiting at a barrier, join a round
// whose window is large, each counting (and ORing) every fourth batch with all
// of a batch's loads in flight (nothing kept in registers between the count and
// the OR, which reloads).  The host launches both; the largest window, found
// while the block maxima are built, decides which one returns at once.
#include <algorithm>
#include <mutex>

#include "common.hpp"

namespace siting {
namespace {

constexpr int kGreedyBlock = 512;    // candidates per bmax entry
constexpr int kGreedyKeys = kGreedyBlock / 64;  // keys of a block per lane
constexpr int kGreedyWords = 16;     // window words per lane per batch
constexpr int kGreedyMaxBlocks = 8192;
#ifndef GREEDY_WAVES
#define GREEDY_WAVES 4
#endif
constexpr int kGreedyWaves = GREEDY_WAVES;  // wavefronts for windows above one batch

// popcount totals of a window: at most (2*16383+1)^2 < 2^31 bits
__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) { return wave_sum_u32((uint32_t)v); }

// A load served by L2, not by the CU's L1: for values this workgroup stored
// earlier in the same launch, where a stale L1 copy would be wrong (with
// intervisibility a key can grow back from 0; a plain key only shrinks, so a
// stale read of it is still an upper bound).
template <typename T>
__device__ __forceinline__ T load_l2(const T *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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

__global__ void greedy_zero(uint64_t *__restrict__ c, int64_t words, uint32_t *__restrict__ maxwords)
{
    if (blockIdx.x == 0 && threadIdx.x == 0)
        *maxwords = 0;
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

// block maxima of the initial keys, one wavefront per block, and the largest
// window (in words) of any valid candidate
__global__ __launch_bounds__(64) void greedy_blocks(const uint64_t *__restrict__ key,
                                                    const int32_t *__restrict__ fresh,
                                                    const siting_observer *__restrict__ obs,
                                                    int64_t n, int64_t nrows, int64_t ncols,
                                                    uint64_t *__restrict__ bmax_g,
                                                    int32_t *__restrict__ bfr_g,
                                                    uint32_t *__restrict__ maxwords)
{
    const int b = blockIdx.x, lane = threadIdx.x;
    uint64_t v;
    int32_t f;
    wave_block_max(key, fresh, n, b, lane, -1, 0, 0, v, f);
    uint32_t mw = 0;
    for (int u = 0; u < kGreedyKeys; u++) {
        const int64_t j = (int64_t)b * kGreedyBlock + u * 64 + lane;
        if (j < n) {
            const siting_observer o = obs[j];
            if (obs_ok(o, nrows, ncols)) {
                const Win w = window_of(o, nrows, ncols);
                mw = max(mw, (uint32_t)(w.rows * w.nw));
            }
        }
    }
    mw = (uint32_t)wave_max_u64(mw);
    if (lane == 0) {
        bmax_g[b] = v;
        bfr_g[b] = f;
        atomicMax(maxwords, mw);
    }
}

// A window (or one wavefront's share of it): words e = eb + k*estep + 64u +
// lane, row-major over the window's rows x nw words.
constexpr int kBatch = 64 * kGreedyWords;

struct Share {
    const uint64_t *v;  // the candidate's window bitmap
    int64_t ylo, w0;    // its first row and first word column in C
    int nw, words;
    int eb, estep;
};

// A window of at most one batch: popcount(V & ~C), the words kept in
// registers for the OR (row and column stepped without division).
__device__ __forceinline__ uint64_t share_count(const Share &s, const uint64_t *C, int64_t W,
                                                int lane, int64_t *cix, uint64_t *vv,
                                                uint64_t *cc)
{
    const int nw1 = s.nw > 0 ? s.nw : 1;
    const int dq = 64 / nw1, dr = 64 - dq * s.nw;
    {
        int row = lane / nw1, col = lane - row * s.nw;
#pragma unroll
        for (int u = 0; u < kGreedyWords; u++) {
            cix[u] = (s.ylo + row) * W + s.w0 + col;
            col += dr;
            row += dq;
            if (col >= s.nw) {
                col -= s.nw;
                row++;
            }
        }
    }
#pragma unroll
    for (int u = 0; u < kGreedyWords; u++) {
        const int e = u * 64 + lane;
        vv[u] = 0;
        cc[u] = 0;
        if (e < s.words) {
            vv[u] = s.v[e];
            cc[u] = C[cix[u]];
        }
    }
    uint64_t cnt = 0;
#pragma unroll
    for (int u = 0; u < kGreedyWords; u++)
        cnt += __popcll(vv[u] & ~cc[u]);
    return cnt;
}

// C |= V for a window of at most one batch, from the registers above
__device__ __forceinline__ void share_or(const Share &s, uint64_t *C, int lane,
                                         const int64_t *cix, const uint64_t *vv,
                                         const uint64_t *cc)
{
#pragma unroll
    for (int u = 0; u < kGreedyWords; u++) {
        const int e = u * 64 + lane;
        if (e < s.words)
            C[cix[u]] = cc[u] | vv[u];
    }
}

// One wavefront's share of a large window (words >= 1), kWords words per
// lane per batch, every load of a batch issued before the first wait: lanes
// past the window's end read its last word and count (or store) nothing.
// Positions advance by estep between batches and by 64 words within one,
// without division.  kStore: C |= V instead of counting.
template <int kWords, bool kStore>
__device__ __forceinline__ uint64_t wide_pass(const Share &s, uint64_t *C, int64_t W, int lane)
{
    const int nw1 = s.nw > 0 ? s.nw : 1;
    const int dq = 64 / nw1, dr = 64 - dq * s.nw;
    const int sq = s.estep / nw1, sr = s.estep - sq * s.nw;
    int row = (s.eb + lane) / nw1, col = s.eb + lane - row * s.nw;
    const int last = s.words - 1;
    const int64_t clast = (s.ylo + last / nw1) * W + s.w0 + (last - (last / nw1) * s.nw);
    uint64_t cnt = 0;
    for (int e0 = s.eb; e0 < s.words; e0 += s.estep) {
        uint64_t v2[kWords], c2[kWords];
        int64_t ix[kWords];
        int r = row, c = col;
#pragma unroll
        for (int u = 0; u < kWords; u++) {
            const bool in = e0 + u * 64 + lane < s.words;
            ix[u] = in ? (s.ylo + r) * W + s.w0 + c : clast;
            v2[u] = s.v[in ? e0 + u * 64 + lane : last];
            c2[u] = C[ix[u]];
            c += dr;
            r += dq;
            if (c >= s.nw) {
                c -= s.nw;
                r++;
            }
        }
#pragma unroll
        for (int u = 0; u < kWords; u++) {
            const bool in = e0 + u * 64 + lane < s.words;
            if (kStore) {
                if (in)
                    C[ix[u]] = c2[u] | v2[u];
            } else {
                cnt += in ? __popcll(v2[u] & ~c2[u]) : 0;
            }
        }
        col += sr;
        row += sq;
        if (col >= s.nw) {
            col -= s.nw;
            row++;
        }
    }
    return cnt;
}

// batch sizes of the large-window passes (words per lane; 32 for the count
// was faster at ROI 1000 but slower at 200 and 500)
constexpr int kWideCount = 16;
constexpr int kWideOr = 16;

// What wavefront 0 tells the helper wavefronts about a large window's round.
struct BigRound {
    int64_t off, ylo, w0, i;  // off: the window's first word in the bitmaps
    uint64_t g, second, bo;
    int nw, words, stale, done;
};

// The selection loop.  Wavefront 0 runs every round; with kWaves > 1 the
// other wavefronts wait at a barrier and join only rounds whose window is
// larger than one batch (64 * kGreedyWords words), each taking every
// kWaves-th batch, so small windows pay no barrier at all.
//
// kInter (intervisibility): after the first pick only candidates whose post
// lies in C compete.  Right after the first pick every other candidate whose
// post C does not cover is parked: its key moves to pbound and becomes 0 (a
// parked key never wins; a stale bound stays an upper bound while it waits),
// and it joins a list of (index, position).  After each later pick, wavefront
// 0 scans that list for parked candidates inside the new window whose post C
// now covers and puts their bounds back (raising the block maxima, marked
// stale).  Eligibility only grows, so each candidate parks at most once.
// Both steps test a post against the window just taken, in the (read-only)
// window bitmap: C was empty before the first pick, and a parked post was
// not in C before the pick that may cover it.
template <int kWaves, bool kInter>
__global__ __launch_bounds__(64 * kWaves) void greedy_run(
    const uint64_t *__restrict__ bitmaps, const int64_t *__restrict__ offsets,
    const siting_observer *__restrict__ obs, int64_t n, int64_t nrows, int64_t ncols,
    int32_t max_obs, int64_t target, uint64_t *C, int64_t *__restrict__ selected,
    int64_t *__restrict__ gains, int32_t *__restrict__ nselected, uint64_t *key, int32_t *fresh,
    const uint64_t *__restrict__ bmax_g, const int32_t *__restrict__ bfr_g,
    const uint32_t *__restrict__ maxwords, uint64_t *__restrict__ pbound,
    int32_t *__restrict__ plist_idx, int64_t *__restrict__ plist_xy)
{
    // both instantiations are launched: one wavefront when every window fits
    // one batch, kWaves otherwise; the other returns at once
    if ((kWaves > 1) != (*maxwords > (uint32_t)kBatch))
        return;
    // block maxima of the keys and the round stamps of those maxima
    extern __shared__ uint64_t bmax[];
    __shared__ uint32_t s_part[kWaves];
    __shared__ BigRound s_big;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t W = (ncols + 63) >> 6;
    const int nblocks = (int)((n + kGreedyBlock - 1) / kGreedyBlock);
    int32_t *bfr = reinterpret_cast<int32_t *>(bmax + nblocks);
    for (int b = threadIdx.x; b < nblocks; b += 64 * kWaves) {
        bmax[b] = bmax_g[b];
        bfr[b] = bfr_g[b];
    }
    __syncthreads();

    if (kWaves > 1 && wave > 0) {
        // ---- helper wavefronts: one large-window round per pass
        for (;;) {
            __syncthreads();  // wavefront 0 has published the round
            const BigRound rb = s_big;
            if (rb.done)
                break;
            // the window's address from the kernel argument, so that its loads
            // stay global loads
            const uint64_t *v = bitmaps + rb.off;
            uint64_t gain = rb.g;
            if (rb.stale) {
                const Share sc{v, rb.ylo, rb.w0, rb.nw, rb.words, wave * 64 * kWideCount,
                               kWaves * 64 * kWideCount};
                const uint64_t cnt = wide_pass<kWideCount, false>(sc, C, W, lane);
                const uint32_t part = (uint32_t)wave_sum_u64(cnt);
                if (lane == 0)
                    s_part[wave] = part;
                __syncthreads();  // every share counted
                uint32_t sum = 0;
#pragma unroll
                for (int q = 0; q < kWaves; q++)
                    sum += s_part[q];
                gain = sum;
            }
            const uint64_t nk = (gain << 32) | (0xFFFFFFFFull - (uint64_t)rb.i);
            const bool take = gain > 0 && (!rb.stale || (nk > rb.second && nk > rb.bo));
            if (take) {
                const Share so{v, rb.ylo, rb.w0, rb.nw, rb.words, wave * 64 * kWideOr,
                               kWaves * 64 * kWideOr};
                wide_pass<kWideOr, true>(so, C, W, lane);
            }
            __syncthreads();  // every share ORed into C
        }
        return;
    }

    // ---- wavefront 0
    int32_t t = 0;
    int64_t covered = 0;
    int64_t nparked = 0;  // entries of the parked list (kInter)
    const uint64_t lt_mask = lane == 0 ? 0ull : (~0ull >> (64 - lane));
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
            if (kInter) {
                kk[u] = j < n && j != skip ? load_l2(&key[j]) : 0;
                ff[u] = j < n ? load_l2(&fresh[j]) : 0;
            } else {
                kk[u] = j < n && j != skip ? key[j] : 0;
                ff[u] = j < n ? fresh[j] : 0;
            }
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
        // the largest key of the top's block other than the top's own (a
        // large window's round needs it before the helpers start, a small
        // one after its window loads are in flight)
        uint64_t bo = 0;
        int32_t fbo = 0;
        auto block_other = [&]() {
            uint64_t kb = 0;
            int32_t fb = 0;
#pragma unroll
            for (int u = 0; u < kGreedyKeys; u++) {
                if (kk[u] > kb) {
                    kb = kk[u];
                    fb = ff[u];
                }
            }
            bo = wave_max_u64(kb);
            const uint64_t bown = __ballot(kb == bo && bo != 0);
            fbo = __builtin_amdgcn_readlane(fb, bown ? __ffsll((long long)bown) - 1 : 0);
        };
        const bool big = kWaves > 1 && words > kBatch;
        if (big) {
            block_other();
            if (lane == 0)
                s_big = BigRound{valid ? off : 0, w.ylo, w.w0, i, g, second, bo, w.nw, words,
                                 stale ? 1 : 0, 0};
            __syncthreads();  // the helpers start
        }
        const Share sh{v, w.ylo, w.w0, w.nw, words, 0, kBatch};
        int64_t cix[kGreedyWords];
        uint64_t vv[kGreedyWords], cc[kGreedyWords];
        uint64_t cnt = 0;
        if (big) {
            if (stale)
                cnt = wide_pass<kWideCount, false>(
                    Share{v, w.ylo, w.w0, w.nw, words, 0, kWaves * 64 * kWideCount}, C, W, lane);
        } else {
            cnt = share_count(sh, C, W, lane, cix, vv, cc);
            block_other();
        }
        uint64_t gain = g;
        if (stale) {
            uint32_t sum = (uint32_t)wave_sum_u64(cnt);
            if (big) {
                if (lane == 0)
                    s_part[0] = sum;
                __syncthreads();  // every share counted
                sum = 0;
#pragma unroll
                for (int q = 0; q < kWaves; q++)
                    sum += s_part[q];
            }
            gain = sum;
        }
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
            if (big)
                wide_pass<kWideOr, true>(
                    Share{v, w.ylo, w.w0, w.nw, words, 0, kWaves * 64 * kWideOr}, C, W, lane);
            else
                share_or(sh, C, lane, cix, vv, cc);
            covered += (int64_t)gain;
            t++;
        }
        if (big)
            __syncthreads();  // the helpers' ORs are in C
        if (kInter && take) {
            // is post (px, py) set in the window just taken?
            const int64_t xlo = o.x - o.roi < 0 ? 0 : o.x - o.roi;
            const int64_t xhi = o.x + o.roi > ncols - 1 ? ncols - 1 : o.x + o.roi;
            const int64_t yhi = w.ylo + w.rows - 1;
            auto in_window = [&](int64_t px, int64_t py) {
                if (px < xlo || px > xhi || py < w.ylo || py > yhi)
                    return false;
                const uint64_t word = v[(py - w.ylo) * w.nw + ((px >> 6) - w.w0)];
                return ((word >> (px & 63)) & 1ull) != 0;
            };
            // this round's stores (keys, stamps) complete before the reads below
            __builtin_amdgcn_s_waitcnt(0);
            if (t == 1) {
                // park every candidate the first window does not cover, block
                // by block (a block's 512 keys are 8 steps of the wavefront),
                // and rebuild the block maxima from the registers
                for (int b = 0; b < nblocks; b++) {
                    uint64_t bv = 0;
                    int32_t bf = 0;
                    for (int u = 0; u < kGreedyKeys; u++) {
                        const int64_t j = (int64_t)b * kGreedyBlock + u * 64 + lane;
                        const bool inb = j < n;
                        const int64_t jj = inb ? j : 0;
                        // every lane loads (lanes past n reload candidate 0 and
                        // discard it), so nothing below is assigned under a branch
                        const siting_observer oj = obs[jj];
                        uint64_t kj = load_l2(&key[jj]);
                        const int32_t fj = load_l2(&fresh[jj]);
                        const bool okj = inb && obs_ok(oj, nrows, ncols);
                        const bool seen = okj && in_window(oj.x, oj.y);
                        const bool out = inb && !seen;  // parked (or invalid): key 0
                        const bool park = okj && !seen;  // invalid records never return
                        if (out) {
                            pbound[j] = kj;
                            key[j] = 0;
                        }
                        kj = out || !inb ? 0 : kj;
                        const int64_t xy = ((int64_t)oj.y << 32) | (uint32_t)oj.x;
                        const uint64_t pm = __ballot(park);
                        if (park) {
                            const int64_t e = nparked + __popcll(pm & lt_mask);
                            plist_idx[e] = (int32_t)j;
                            plist_xy[e] = xy;
                        }
                        nparked += __popcll(pm);
                        if (kj > bv) {
                            bv = kj;
                            bf = fj;
                        }
                    }
                    const uint64_t m = wave_max_u64(bv);
                    const uint64_t own = __ballot(bv == m && m != 0);
                    const int32_t mf =
                        __builtin_amdgcn_readlane(bf, own ? __ffsll((long long)own) - 1 : 0);
                    if (lane == 0) {
                        bmax[b] = m;
                        bfr[b] = mf;
                    }
                }
            } else {
                // parked candidates whose post the window just taken covers
                // become eligible again with their old bound
                for (int64_t e0 = 0; e0 < nparked; e0 += 64) {
                    const int64_t e = e0 + lane;
                    if (e >= nparked)
                        continue;
                    const int64_t xy = load_l2(&plist_xy[e]);
                    const int64_t px = (int64_t)(int32_t)(uint32_t)xy, py = xy >> 32;
                    if (!in_window(px, py))
                        continue;
                    const int32_t j = load_l2(&plist_idx[e]);
                    if (j < 0)
                        continue;
                    const uint64_t kj = load_l2(&pbound[j]);
                    key[j] = kj;
                    plist_idx[e] = -1;
                    const int b = j / kGreedyBlock;
                    const uint64_t old = atomicMax(reinterpret_cast<unsigned long long *>(&bmax[b]),
                                                   (unsigned long long)kj);
                    if (kj > old)
                        bfr[b] = -1;  // the block's maximum is a stale bound now
                }
            }
            // the keys and list entries stored above complete before the
            // next round reads them
            __builtin_amdgcn_s_waitcnt(0);
        }
        // the next top: the best key outside block bi or bi's new maximum
        if (kInter && take) {
            pf_i = -1;  // keys of many blocks may have changed: no prefetch
        } else {
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
        // one wavefront's LDS accesses run in order: this only keeps the
        // compiler from moving them across rounds (with helpers waiting at
        // the barrier, wavefront 0 alone must not arrive there)
        if (kWaves == 1)
            __syncthreads();
        else
            __asm__ volatile("" ::: "memory");
    }
    if (kWaves > 1) {
        if (lane == 0)
            s_big.done = 1;
        __syncthreads();  // the helpers leave
    }
    if (lane == 0)
        *nselected = t;
}

// ---------------------------------------------------------------------------
// SITE for large windows, rounds spread over the GPU (host-driven).  The same
// lazy greedy and the same selection: in every round a set S of candidates
// (the top candidate of the top block, then of the blocks whose maxima carry
// the m largest gain bounds) is re-evaluated by one workgroup each, in
// parallel, and then the largest key overall is taken if it is fresh (a fresh
// key at least every stale bound is the plain greedy choice).  A stale top
// after the evaluation is in the next round's S, so every round either selects
// or makes a stale top exact.  Device state: key, fresh, bmax, bfr as in the
// one-workgroup kernel, plus the round control below.
constexpr int kParMax = 1024;  // largest S

struct ParCtl {
    int32_t t;           // observers selected so far
    int32_t done;        // the run has ended (every later kernel returns)
    int32_t or_pending;  // this round selected sel_i, whose window still goes into C
    int32_t nS;          // entries of S this round
    int64_t covered;
    int64_t sel_i;
};

__global__ void gpar_init(ParCtl *ctl, int32_t max_obs, int64_t target)
{
    ctl->t = 0;
    ctl->done = (max_obs <= 0 || target <= 0) ? 1 : 0;
    ctl->or_pending = 0;
    ctl->nS = 0;
    ctl->covered = 0;
    ctl->sel_i = -1;
}

// S for this round: the top block first, then blocks whose maximum's gain
// exceeds theta, then blocks at theta, at most m; theta is the m-th largest
// gain among the non-empty block maxima (radix selection over its 4 bytes).
__global__ __launch_bounds__(1024) void gpar_select(const uint64_t *__restrict__ bmax, int nb,
                                                   ParCtl *ctl, int64_t *__restrict__ S_cand,
                                                   int32_t *__restrict__ S_blk, int m)
{
    __shared__ uint32_t hist[256];
    __shared__ uint32_t s_prefix, s_mask, s_rem, s_count, s_nz;
    __shared__ uint64_t s_wmax[16];
    __shared__ int s_topb;
    if (ctl->done)
        return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    uint64_t mk = 0;
    uint32_t nz = 0;
    for (int b = tid; b < nb; b += 1024) {
        const uint64_t v = bmax[b];
        mk = v > mk ? v : mk;
        nz += v != 0;
    }
    mk = wave_max_u64(mk);
    nz = wave_sum_u32(nz);
    if (tid == 0) {
        s_nz = 0;
        s_prefix = 0;
        s_mask = 0;
        s_rem = (uint32_t)m;
    }
    __syncthreads();
    if (lane == 0) {
        s_wmax[wave] = mk;
        atomicAdd(&s_nz, nz);
    }
    __syncthreads();
    uint64_t top = 0;
#pragma unroll
    for (int w = 0; w < 16; w++)
        top = s_wmax[w] > top ? s_wmax[w] : top;
    const uint32_t nonzero = s_nz;
    if (top == 0) {
        if (tid == 0)
            ctl->nS = 0;
        return;
    }
    const int64_t top_i = (int64_t)(0xFFFFFFFFull - (top & 0xFFFFFFFFull));
    uint32_t theta = 0;
    if (nonzero > (uint32_t)m) {
        for (int pass = 0; pass < 4; pass++) {
            const int shift = 24 - 8 * pass;
            if (tid < 256)
                hist[tid] = 0;
            __syncthreads();
            const uint32_t pre = s_prefix, msk = s_mask;
            for (int b = tid; b < nb; b += 1024) {
                const uint64_t v = bmax[b];
                const uint32_t g = (uint32_t)(v >> 32);
                if (v != 0 && (g & msk) == pre)
                    atomicAdd(&hist[(g >> shift) & 0xFFu], 1u);
            }
            __syncthreads();
            if (tid == 0) {
                uint32_t cum = 0, rem = s_rem;
                int sel = 0;
                for (int d = 255; d >= 0; d--) {
                    if (cum + hist[d] >= rem) {
                        sel = d;
                        rem -= cum;
                        break;
                    }
                    cum += hist[d];
                }
                s_rem = rem;
                s_prefix = pre | ((uint32_t)sel << shift);
                s_mask = msk | (0xFFu << shift);
            }
            __syncthreads();
        }
        theta = s_prefix;
    }
    if (tid == 0) {
        s_topb = (int)(top_i / kGreedyBlock);
        s_count = 1;
        S_blk[0] = s_topb;
        S_cand[0] = top_i;
    }
    __syncthreads();
    const int topb = s_topb;
    for (int phase = 0; phase < 2; phase++) {
        for (int b = tid; b < nb; b += 1024) {
            const uint64_t v = bmax[b];
            const uint32_t g = (uint32_t)(v >> 32);
            if (v == 0 || b == topb || (phase == 0 ? g <= theta : g != theta))
                continue;
            const uint32_t slot = atomicAdd(&s_count, 1u);
            if (slot < (uint32_t)m) {
                S_blk[slot] = b;
                S_cand[slot] = (int64_t)(0xFFFFFFFFull - (v & 0xFFFFFFFFull));
            }
        }
        __syncthreads();
    }
    if (tid == 0)
        ctl->nS = (int)(s_count < (uint32_t)m ? s_count : (uint32_t)m);
}

// One workgroup per entry of S: a stale candidate's gain |V \ C| afresh, then
// its block's maximum (every block appears in S at most once).
__global__ __launch_bounds__(256) void gpar_eval(
    const uint64_t *__restrict__ bitmaps, const int64_t *__restrict__ offsets,
    const siting_observer *__restrict__ obs, int64_t n, int64_t nrows, int64_t ncols,
    const uint64_t *__restrict__ C, uint64_t *key, int32_t *fresh, const ParCtl *ctl,
    const int64_t *__restrict__ S_cand, const int32_t *__restrict__ S_blk, uint64_t *bmax,
    int32_t *bfr)
{
    __shared__ uint32_t s_part[4];
    if (ctl->done || (int)blockIdx.x >= ctl->nS)
        return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int32_t t = ctl->t;
    const int64_t i = S_cand[blockIdx.x];
    const int b = S_blk[blockIdx.x];
    uint64_t ki = 0;
    int32_t fi = 0;
    bool over = false;
    if (fresh[i] != t) {
        const siting_observer o = obs[i];
        uint32_t cnt = 0;
        if (obs_ok(o, nrows, ncols)) {
            const Win w = window_of(o, nrows, ncols);
            const uint64_t *v = bitmaps + offsets[i];
            const int64_t W = (ncols + 63) >> 6;
            const int words = w.rows * w.nw;
            // four words per thread in flight; row and column by division
            for (int e0 = 0; e0 < words; e0 += 1024) {
                uint64_t vv[4], cc[4];
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    const int e = e0 + u * 256 + tid;
                    vv[u] = 0;
                    cc[u] = 0;
                    if (e < words) {
                        const int r = e / w.nw, c = e - r * w.nw;
                        vv[u] = v[e];
                        cc[u] = C[(w.ylo + r) * W + w.w0 + c];
                    }
                }
#pragma unroll
                for (int u = 0; u < 4; u++)
                    cnt += (uint32_t)__popcll(vv[u] & ~cc[u]);
            }
        }
        cnt = wave_sum_u32(cnt);
        if (lane == 0)
            s_part[wave] = cnt;
        __syncthreads();
        const uint64_t gain = (uint64_t)s_part[0] + s_part[1] + s_part[2] + s_part[3];
        ki = (gain << 32) | (0xFFFFFFFFull - (uint64_t)i);
        fi = t;
        over = true;
        if (tid == 0) {
            key[i] = ki;
            fresh[i] = fi;
        }
    }
    if (wave == 0) {
        uint64_t v;
        int32_t f;
        // the new key of i is taken from registers, not read back
        wave_block_max(key, fresh, n, b, lane, over ? i : -1, ki, fi, v, f);
        if (lane == 0) {
            bmax[b] = v;
            bfr[b] = f;
        }
    }
}

// The round's decision (one workgroup): the largest key overall; a fresh one
// is selected (a zero gain or an exhausted key set ends the run).
__global__ __launch_bounds__(1024) void gpar_decide(
    uint64_t *key, int32_t *fresh, uint64_t *bmax, int32_t *bfr, int nb, int64_t n,
    int32_t max_obs, int64_t target, ParCtl *ctl, int64_t *__restrict__ selected,
    int64_t *__restrict__ gains)
{
    __shared__ uint64_t s_wmax[16];
    if (ctl->done)
        return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    uint64_t mk = 0;
    for (int b = tid; b < nb; b += 1024) {
        const uint64_t v = bmax[b];
        mk = v > mk ? v : mk;
    }
    mk = wave_max_u64(mk);
    if (lane == 0)
        s_wmax[wave] = mk;
    __syncthreads();
    uint64_t top = 0;
#pragma unroll
    for (int w = 0; w < 16; w++)
        top = s_wmax[w] > top ? s_wmax[w] : top;
    const int32_t t = ctl->t;
    const int64_t i = (int64_t)(0xFFFFFFFFull - (top & 0xFFFFFFFFull));
    const uint64_t g = top >> 32;
    const int bi = (int)(i / kGreedyBlock);
    const bool stale = top != 0 && bfr[bi] != t;
    const bool end = top == 0 || i >= n || (!stale && g == 0);
    const bool take = !end && !stale;
    if (wave == 0) {
        if (take) {
            // i's key drops to a zero gain, fresh from now on; its block's maximum
            const uint64_t ki = 0xFFFFFFFFull - (uint64_t)i;
            uint64_t v;
            int32_t f;
            wave_block_max(key, fresh, n, bi, lane, i, ki, t + 1, v, f);
            if (lane == 0) {
                key[i] = ki;
                fresh[i] = t + 1;
                bmax[bi] = v;
                bfr[bi] = f;
                selected[t] = i;
                gains[t] = (int64_t)g;
                const int64_t cov = ctl->covered + (int64_t)g;
                ctl->covered = cov;
                ctl->sel_i = i;
                ctl->or_pending = 1;
                ctl->t = t + 1;
                ctl->done = (t + 1 >= max_obs || cov >= target) ? 1 : 0;
            }
        } else if (lane == 0) {
            ctl->or_pending = 0;
            if (end)
                ctl->done = 1;
        }
    }
}

// C |= V of the observer selected this round, spread over the grid.
__global__ __launch_bounds__(256) void gpar_or(const uint64_t *__restrict__ bitmaps,
                                               const int64_t *__restrict__ offsets,
                                               const siting_observer *__restrict__ obs,
                                               int64_t nrows, int64_t ncols, uint64_t *C,
                                               const ParCtl *ctl)
{
    if (!ctl->or_pending)
        return;
    const int64_t i = ctl->sel_i;
    const siting_observer o = obs[i];
    const Win w = window_of(o, nrows, ncols);
    const uint64_t *v = bitmaps + offsets[i];
    const int64_t W = (ncols + 63) >> 6;
    const int words = w.rows * w.nw;
    for (int e = blockIdx.x * 256 + threadIdx.x; e < words; e += gridDim.x * 256) {
        const int r = e / w.nw, c = e - r * w.nw;
        C[(w.ylo + r) * W + w.w0 + c] |= v[e];
    }
}

__global__ void gpar_finish(const ParCtl *ctl, int32_t *nselected) { *nselected = ctl->t; }

}  // namespace
}  // namespace siting

using namespace siting;

static constexpr size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Workspace layout of n candidates: key[n] u64, fresh[n] i32, block maxima
// bmax[nb] u64 and their stamps bfr[nb] i32, the largest window's words u32;
// with intervisibility also the parked bounds pbound[n] u64 and the parked
// list (index i32, packed position i64) of up to n entries.
static constexpr size_t greedy_ws_bytes(int64_t n)
{
    return align256((size_t)n * 8) + align256((size_t)n * 4) +
           align256((size_t)((n + kGreedyBlock - 1) / kGreedyBlock) * 8) +
           align256((size_t)((n + kGreedyBlock - 1) / kGreedyBlock) * 4) + align256(4);
}
static constexpr size_t greedy_inter_ws_bytes(int64_t n)
{
    return greedy_ws_bytes(n) + align256((size_t)n * 8) + align256((size_t)n * 4) +
           align256((size_t)n * 8);
}
// The parallel-round path: the round control and the set S after the
// one-workgroup layout.
static constexpr size_t greedy_par_ws_bytes(int64_t n)
{
    return greedy_ws_bytes(n) + align256(sizeof(ParCtl)) + align256((size_t)kParMax * 8) +
           align256((size_t)kParMax * 4);
}

// The allocation-free entry point keeps its workspace in this array (one
// copy per device, held until the process ends).  Host code must not pass
// the array's name to a kernel: it is a host-side stand-in, and the device
// address comes from hipGetSymbolAddress (noalloc_scratch below).
constexpr int64_t kNoAllocMaxN = SITING_GREEDY_NOALLOC_MAX_N;
constexpr size_t kNoAllocBytes = greedy_ws_bytes(kNoAllocMaxN);
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

extern "C" size_t siting_greedy_workspace_size(int64_t n)
{
    if (n < 0)
        return 0;
    // enough for every entry point
    return std::max(greedy_inter_ws_bytes(n), greedy_par_ws_bytes(n));
}

// Argument validation shared by both entry points (host only); SITING_OK or
// an error code.
static int greedy_check(const char *fn, const uint64_t *bitmaps, const int64_t *offsets,
                        const siting_observer *obs, int64_t n, int64_t nrows, int64_t ncols,
                        int32_t max_obs, const uint64_t *cumulative, const int64_t *selected,
                        const int64_t *gains, const int32_t *nselected)
{
    SITING_REQUIRE(n >= 1 && n < 0xFFFFFFFFll, "%s: n must be in 1..2^32-2", fn);
    SITING_REQUIRE(nrows >= 1 && ncols >= 1, "%s: empty terrain", fn);
    SITING_REQUIRE(max_obs >= 0, "%s: max_obs < 0", fn);
    SITING_REQUIRE(bitmaps && offsets && obs && cumulative && nselected,
                   "%s: NULL device pointer", fn);
    SITING_REQUIRE(max_obs == 0 || (selected && gains), "%s: NULL selected/gains", fn);
    return SITING_OK;
}

// The candidate count the block maxima in LDS allow (asks the device).
static int greedy_limits(const char *fn, int64_t n)
{
    const int64_t nblocks = (n + kGreedyBlock - 1) / kGreedyBlock;
    const int lds_max = std::min(
        std::min(kernel_max_dynamic_lds(reinterpret_cast<const void *>(&greedy_run<1, false>)),
                 kernel_max_dynamic_lds(
                     reinterpret_cast<const void *>(&greedy_run<kGreedyWaves, false>))),
        std::min(kernel_max_dynamic_lds(reinterpret_cast<const void *>(&greedy_run<1, true>)),
                 kernel_max_dynamic_lds(
                     reinterpret_cast<const void *>(&greedy_run<kGreedyWaves, true>))));
    if (nblocks > kGreedyMaxBlocks || nblocks * 12 > lds_max) {
        set_error("%s: %lld candidates exceed the supported maximum", fn, (long long)n);
        return SITING_E_UNSUPPORTED;
    }
    return SITING_OK;
}

// Enqueues the rounds on `ws` (greedy_ws_bytes(n) bytes of device memory,
// greedy_inter_ws_bytes(n) with intervisibility; every part is written
// before it is read, so it needs no clearing).
static int greedy_launch(const uint64_t *bitmaps, const int64_t *offsets,
                         const siting_observer *obs, int64_t n, int64_t nrows, int64_t ncols,
                         int32_t max_obs, int64_t target_cells, uint64_t *cumulative,
                         int64_t *selected, int64_t *gains, int32_t *nselected, void *ws,
                         void *stream, bool inter)
{
    const int64_t nblocks = (n + kGreedyBlock - 1) / kGreedyBlock;
    char *wsb = reinterpret_cast<char *>(ws);
    uint64_t *key = reinterpret_cast<uint64_t *>(wsb);
    wsb += align256((size_t)n * 8);
    int32_t *fresh = reinterpret_cast<int32_t *>(wsb);
    wsb += align256((size_t)n * 4);
    uint64_t *bmax_g = reinterpret_cast<uint64_t *>(wsb);
    wsb += align256((size_t)nblocks * 8);
    int32_t *bfr_g = reinterpret_cast<int32_t *>(wsb);
    wsb += align256((size_t)nblocks * 4);
    uint32_t *maxwords = reinterpret_cast<uint32_t *>(wsb);
    wsb += align256(4);
    uint64_t *pbound = nullptr;
    int32_t *plist_idx = nullptr;
    int64_t *plist_xy = nullptr;
    if (inter) {
        pbound = reinterpret_cast<uint64_t *>(wsb);
        wsb += align256((size_t)n * 8);
        plist_idx = reinterpret_cast<int32_t *>(wsb);
        wsb += align256((size_t)n * 4);
        plist_xy = reinterpret_cast<int64_t *>(wsb);
    }
    hipStream_t s = as_stream(stream);
    const int64_t W = (ncols + 63) / 64;
    const int64_t cwords = nrows * W;
    const int zg = (int)std::min<int64_t>((cwords + 255) / 256, (int64_t)device_cus() * 16);
    int rc;
    hipLaunchKernelGGL(greedy_zero, dim3(zg > 0 ? zg : 1), dim3(256), 0, s, cumulative, cwords,
                       maxwords);
    if ((rc = check_launch("greedy_zero")) != SITING_OK)
        return rc;
    hipLaunchKernelGGL(greedy_init, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, bitmaps,
                       offsets, obs, n, nrows, ncols, key, fresh);
    if ((rc = check_launch("greedy_init")) != SITING_OK)
        return rc;
    hipLaunchKernelGGL(greedy_blocks, dim3((unsigned)nblocks), dim3(64), 0, s, key, fresh, obs, n,
                       nrows, ncols, bmax_g, bfr_g, maxwords);
    if ((rc = check_launch("greedy_blocks")) != SITING_OK)
        return rc;
    // one of the two returns at once (the largest window decides)
#define GREEDY_RUN(WAVES, INTER)                                                                \
    hipLaunchKernelGGL((greedy_run<WAVES, INTER>), dim3(1), dim3(64 * (WAVES)),                \
                       (size_t)nblocks * 12, s, bitmaps, offsets, obs, n, nrows, ncols, max_obs, \
                       target_cells, cumulative, selected, gains, nselected, key, fresh, bmax_g, \
                       bfr_g, maxwords, pbound, plist_idx, plist_xy)
    if (inter)
        GREEDY_RUN(1, true);
    else
        GREEDY_RUN(1, false);
    if ((rc = check_launch("greedy_run")) != SITING_OK)
        return rc;
    if (inter)
        GREEDY_RUN(kGreedyWaves, true);
    else
        GREEDY_RUN(kGreedyWaves, false);
#undef GREEDY_RUN
    return check_launch("greedy_run");
}

extern "C" int siting_greedy(const uint64_t *bitmaps, const int64_t *offsets,
                             const siting_observer *obs, int64_t n, int64_t nrows, int64_t ncols,
                             int32_t max_obs, int64_t target_cells, uint64_t *cumulative,
                             int64_t *selected, int64_t *gains, int32_t *nselected, void *ws,
                             size_t ws_bytes, void *stream)
{
    clear_error();
    const char *fn = "siting_greedy";
    int rc = greedy_check(fn, bitmaps, offsets, obs, n, nrows, ncols, max_obs, cumulative,
                          selected, gains, nselected);
    if (rc != SITING_OK)
        return rc;
    const size_t need = greedy_ws_bytes(n);
    if (ws == nullptr || ws_bytes < need) {
        set_error("%s: workspace of %zu bytes needed", fn, need);
        return SITING_E_WORKSPACE;
    }
    if ((rc = greedy_limits(fn, n)) != SITING_OK)
        return rc;
    return greedy_launch(bitmaps, offsets, obs, n, nrows, ncols, max_obs, target_cells,
                         cumulative, selected, gains, nselected, ws, stream, false);
}

extern "C" int siting_greedy_intervisible(const uint64_t *bitmaps, const int64_t *offsets,
                                          const siting_observer *obs, int64_t n, int64_t nrows,
                                          int64_t ncols, int32_t max_obs, int64_t target_cells,
                                          uint64_t *cumulative, int64_t *selected,
                                          int64_t *gains, int32_t *nselected, void *ws,
                                          size_t ws_bytes, void *stream)
{
    clear_error();
    const char *fn = "siting_greedy_intervisible";
    int rc = greedy_check(fn, bitmaps, offsets, obs, n, nrows, ncols, max_obs, cumulative,
                          selected, gains, nselected);
    if (rc != SITING_OK)
        return rc;
    const size_t need = greedy_inter_ws_bytes(n);
    if (ws == nullptr || ws_bytes < need) {
        set_error("%s: workspace of %zu bytes needed", fn, need);
        return SITING_E_WORKSPACE;
    }
    if ((rc = greedy_limits(fn, n)) != SITING_OK)
        return rc;
    return greedy_launch(bitmaps, offsets, obs, n, nrows, ncols, max_obs, target_cells,
                         cumulative, selected, gains, nselected, ws, stream, true);
}

extern "C" int siting_greedy_parallel(const uint64_t *bitmaps, const int64_t *offsets,
                                      const siting_observer *obs, int64_t n, int64_t nrows,
                                      int64_t ncols, int32_t max_obs, int64_t target_cells,
                                      int32_t batch, uint64_t *cumulative, int64_t *selected,
                                      int64_t *gains, int32_t *nselected, void *ws,
                                      size_t ws_bytes, void *stream)
{
    clear_error();
    const char *fn = "siting_greedy_parallel";
    int rc = greedy_check(fn, bitmaps, offsets, obs, n, nrows, ncols, max_obs, cumulative,
                          selected, gains, nselected);
    if (rc != SITING_OK)
        return rc;
    SITING_REQUIRE(batch >= 1 && batch <= kParMax, "%s: batch %d outside 1..%d", fn, batch,
                   kParMax);
    SITING_REQUIRE(n <= (int64_t)kGreedyMaxBlocks * kGreedyBlock,
                   "%s: %lld candidates above the supported maximum", fn, (long long)n);
    const size_t need = greedy_par_ws_bytes(n);
    if (ws == nullptr || ws_bytes < need) {
        set_error("%s: workspace of %zu bytes needed", fn, need);
        return SITING_E_WORKSPACE;
    }
    const int nb = (int)((n + kGreedyBlock - 1) / kGreedyBlock);
    char *wsb = reinterpret_cast<char *>(ws);
    uint64_t *key = reinterpret_cast<uint64_t *>(wsb);
    wsb += align256((size_t)n * 8);
    int32_t *fresh = reinterpret_cast<int32_t *>(wsb);
    wsb += align256((size_t)n * 4);
    uint64_t *bmax = reinterpret_cast<uint64_t *>(wsb);
    wsb += align256((size_t)nb * 8);
    int32_t *bfr = reinterpret_cast<int32_t *>(wsb);
    wsb += align256((size_t)nb * 4);
    uint32_t *maxwords = reinterpret_cast<uint32_t *>(wsb);
    wsb += align256(4);
    ParCtl *ctl = reinterpret_cast<ParCtl *>(wsb);
    wsb += align256(sizeof(ParCtl));
    int64_t *S_cand = reinterpret_cast<int64_t *>(wsb);
    wsb += align256((size_t)kParMax * 8);
    int32_t *S_blk = reinterpret_cast<int32_t *>(wsb);
    hipStream_t s = as_stream(stream);
    const int64_t W = (ncols + 63) / 64;
    const int64_t cwords = nrows * W;
    const int cus = device_cus();
    const int zg = (int)std::min<int64_t>((cwords + 255) / 256, (int64_t)cus * 16);
    hipLaunchKernelGGL(greedy_zero, dim3(zg > 0 ? zg : 1), dim3(256), 0, s, cumulative, cwords,
                       maxwords);
    if ((rc = check_launch("greedy_zero")) != SITING_OK)
        return rc;
    hipLaunchKernelGGL(greedy_init, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, bitmaps,
                       offsets, obs, n, nrows, ncols, key, fresh);
    if ((rc = check_launch("greedy_init")) != SITING_OK)
        return rc;
    hipLaunchKernelGGL(greedy_blocks, dim3((unsigned)nb), dim3(64), 0, s, key, fresh, obs, n,
                       nrows, ncols, bmax, bfr, maxwords);
    if ((rc = check_launch("greedy_blocks")) != SITING_OK)
        return rc;
    hipLaunchKernelGGL(gpar_init, dim3(1), dim3(1), 0, s, ctl, max_obs, target_cells);
    if ((rc = check_launch("gpar_init")) != SITING_OK)
        return rc;
    // rounds are enqueued in growing batches; every kernel of a round after
    // the end returns at once.  Each round selects or makes a stale top exact,
    // so at most (n + 1) rounds pass between two selections.
    const int64_t max_rounds = ((int64_t)max_obs + 1) * (n + 1);
    int64_t rounds = 0;
    int chunk = 32;
    for (;;) {
        for (int r = 0; r < chunk; r++) {
            hipLaunchKernelGGL(gpar_select, dim3(1), dim3(1024), 0, s, bmax, nb, ctl, S_cand,
                               S_blk, (int)batch);
            hipLaunchKernelGGL(gpar_eval, dim3((unsigned)batch), dim3(256), 0, s, bitmaps, offsets,
                               obs, n, nrows, ncols, cumulative, key, fresh, ctl, S_cand, S_blk,
                               bmax, bfr);
            hipLaunchKernelGGL(gpar_decide, dim3(1), dim3(1024), 0, s, key, fresh, bmax, bfr, nb,
                               n, max_obs, target_cells, ctl, selected, gains);
            hipLaunchKernelGGL(gpar_or, dim3((unsigned)(cus * 2)), dim3(256), 0, s, bitmaps,
                               offsets, obs, nrows, ncols, cumulative, ctl);
        }
        if ((rc = check_launch("gpar round")) != SITING_OK)
            return rc;
        rounds += chunk;
        int32_t done = 0;
        SITING_HIP(hipMemcpyAsync(&done, &ctl->done, sizeof(done), hipMemcpyDeviceToHost, s));
        SITING_HIP(hipStreamSynchronize(s));
        if (done)
            break;
        if (rounds > max_rounds) {
            set_error("%s: no end after %lld rounds", fn, (long long)rounds);
            return SITING_E_INTERNAL;
        }
        chunk = std::min(chunk * 2, 512);
    }
    hipLaunchKernelGGL(gpar_finish, dim3(1), dim3(1), 0, s, ctl, nselected);
    return check_launch("gpar_finish");
}

// Device address of `scratch` on the current device, looked up once per
// device (each device holds its own copy of the array at its own address).
static int noalloc_scratch(const char *fn, void **out)
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        set_error("%s: hipGetDevice failed: %s", fn, hipGetErrorString(e));
        return SITING_E_HIP;
    }
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("%s: device %d beyond the supported %d", fn, dev, kMaxDevices);
        return SITING_E_UNSUPPORTED;
    }
    std::lock_guard<std::mutex> lock(mu);
    if (addr[dev] == nullptr) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr) {
            set_error("%s: hipGetSymbolAddress(scratch) failed: %s", fn, hipGetErrorString(e));
            return SITING_E_HIP;
        }
        addr[dev] = p;
    }
    *out = addr[dev];
    return SITING_OK;
}

extern "C" int siting_greedy_noalloc(const uint64_t *bitmaps, const int64_t *offsets,
                                     const siting_observer *obs, int64_t n, int64_t nrows,
                                     int64_t ncols, int32_t max_obs, int64_t target_cells,
                                     uint64_t *cumulative, int64_t *selected, int64_t *gains,
                                     int32_t *nselected, void *stream)
{
    clear_error();
    const char *fn = "siting_greedy_noalloc";
    int rc = greedy_check(fn, bitmaps, offsets, obs, n, nrows, ncols, max_obs, cumulative,
                          selected, gains, nselected);
    if (rc != SITING_OK)
        return rc;
    if (n > kNoAllocMaxN) {
        set_error("%s: %lld candidates above the maximum %lld of the static workspace", fn,
                  (long long)n, (long long)kNoAllocMaxN);
        return SITING_E_UNSUPPORTED;
    }
    if ((rc = greedy_limits(fn, n)) != SITING_OK)
        return rc;
    void *ws = nullptr;
    if ((rc = noalloc_scratch(fn, &ws)) != SITING_OK)
        return rc;
    return greedy_launch(bitmaps, offsets, obs, n, nrows, ncols, max_obs, target_cells,
                         cumulative, selected, gains, nselected, ws, stream, false);
}
