// FINDMAX: the k best posts of every block of a grid_r x grid_c block grid
// (stage Findmax: blocks of width ROI/3, 20 transmitters kept per block).
//
// One workgroup per block.  Each post becomes one unique 64-bit key, larger
// is better:
//   u8 keys : count << 56 | (z ^ 0x8000) << 40 | (2^40-1 - local)
//   f32 keys: ord(score) << 32 | (2^32-1 - local)
// where local is the row-major index inside the block (same order as the
// global linear index) and ord() maps floats to order-preserving unsigned
// integers (NaN as -infinity).  f32 keys score the cells of a stride grid;
// a winning cell is returned as its highest post.
// Every wavefront keeps its best k keys sorted across its lanes (lane i holds
// the i-th) and streams its share of the block; a ballot against the
// threshold (the larger of its own k-th key and the best k-th key any
// wavefront has published in LDS) finds the rare candidates, each inserted by
// one shift of the list across lanes.  The wavefronts' lists are then merged
// by k rounds of a workgroup argmax.
// HBM-bound: 3 bytes per post (u8 key + int16 z), read once, coalesced; with
// 16-byte aligned rows each lane streams 16 posts per step in 16-byte loads.
#include "common.hpp"

namespace siting {
namespace {

constexpr int kFmThreads = 256;
constexpr int kFmMaxK = 32;

__device__ __forceinline__ uint32_t ord_f32(float f)
{
    uint32_t b = __float_as_uint(f);
    if (f != f)
        b = 0xFF800000u;  // NaN ranks as -infinity
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

// kVec (u8 keys only): key rows and terrain rows start 16-byte aligned, and
// every lane streams 16 posts per step with three 16-byte loads.
template <bool kF32, bool kVec>
__global__ __launch_bounds__(kFmThreads) void findmax_kernel(
    const void *__restrict__ keyp, int stride, const int16_t *__restrict__ z, int64_t nrows,
    int64_t ncols, int64_t ld, int grid_r, int grid_c, int k, int64_t *__restrict__ cand)
{
    __shared__ uint64_t wmax[kFmThreads / 64];
    // largest k-th best key of any wavefront's list: the block has at least k
    // keys at or above it, so no key below it can be among the block's k best
    __shared__ unsigned long long s_thr;
    int64_t blk = blockIdx.x;
    int bi = (int)(blk / grid_c), bj = (int)(blk % grid_c);
    int64_t r0 = (int64_t)bi * nrows / grid_r, r1 = (int64_t)(bi + 1) * nrows / grid_r;
    int64_t c0 = (int64_t)bj * ncols / grid_c, c1 = (int64_t)(bj + 1) * ncols / grid_c;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    if (tid == 0)
        s_thr = 0;
    __syncthreads();
    // The wavefront's best k keys, sorted across lanes: lane i < k holds the
    // i-th best (0 = none yet; 0 is below every valid key), lanes >= k hold 0.
    uint64_t T = 0;
    uint64_t thr = 0;        // wavefront-uniform: max(own k-th best, shared)
    uint64_t published = 0;  // the largest value this wavefront sent to s_thr
    // Every lane offers one key (0 for none), all lanes together: candidates
    // above the threshold are inserted one at a time (a shift of the list
    // across lanes), the threshold rising as they go.
    auto offer = [&](uint64_t key) {
        uint64_t m = __ballot(key > thr);
        while (m) {
            const int src = __ffsll((long long)m) - 1;
            m &= m - 1;
            const uint64_t kk = __shfl(key, src, 64);
            if (kk > thr) {
                const uint64_t prev = __shfl_up(T, 1, 64);
                const uint64_t nt = T > kk ? T : ((lane == 0 || prev > kk) ? kk : prev);
                T = lane < k ? nt : 0;
                const uint64_t own = __shfl(T, k - 1, 64);
                thr = own > thr ? own : thr;
            }
        }
    };
    auto sync_thr = [&]() {
        if (thr > published) {
            if (lane == 0)
                __hip_atomic_fetch_max(&s_thr, (unsigned long long)thr, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
            published = thr;
        }
        const uint64_t sh =
            __hip_atomic_load(&s_thr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        thr = sh > thr ? sh : thr;
    };
    int64_t lr0, lr1, lc0, lc1;  // rows/cols of the key lattice inside the block
    if (!kF32) {
        lr0 = r0; lr1 = r1; lc0 = c0; lc1 = c1;
    } else {
        lr0 = (r0 + stride - 1) / stride; lr1 = (r1 + stride - 1) / stride;
        lc0 = (c0 + stride - 1) / stride; lc1 = (c1 + stride - 1) / stride;
    }
    int64_t bw = lc1 - lc0, bh = lr1 - lr0;
    int64_t kc = kF32 ? (ncols + stride - 1) / stride : ncols;
    if (kVec) {
        // the wavefront walks (row, 16-post chunk) pairs of the block, 64 at
        // a time; a post's key is built only when its (count, elevation)
        // reaches the threshold's
        const int64_t cc0 = c0 & ~15ll;
        const uint32_t nch = (uint32_t)((((c1 + 15) & ~15ll) - cc0) >> 4);
        const uint32_t total = (uint32_t)bh * nch;
        for (uint32_t i0 = (uint32_t)wave * 64; i0 < total; i0 += kFmThreads) {
            sync_thr();
            const uint32_t i = i0 + lane;
            const bool live = i < total;
            const uint32_t ii = live ? i : i0;  // a valid chunk for idle lanes
            const uint32_t row = ii / nch, ch = ii - row * nch;
            const int64_t ly = r0 + row;
            const int64_t cb = cc0 + ((int64_t)ch << 4);
            const uint4 kv = *reinterpret_cast<const uint4 *>((const uint8_t *)keyp + ly * ncols + cb);
            const uint4 za = *reinterpret_cast<const uint4 *>(z + ly * ld + cb);
            const uint4 zb = *reinterpret_cast<const uint4 *>(z + ly * ld + cb + 8);
            const uint32_t kw[4] = {kv.x, kv.y, kv.z, kv.w};
            const uint32_t zw[8] = {za.x, za.y, za.z, za.w, zb.x, zb.y, zb.z, zb.w};
            const uint64_t lbase = (uint64_t)row * (uint64_t)bw + (uint64_t)(cb - c0);
#pragma unroll
            for (int q = 0; q < 16; q++) {
                const uint32_t c = (kw[q >> 2] >> ((q & 3) * 8)) & 0xFFu;
                const uint32_t zz = ((zw[q >> 1] >> ((q & 1) * 16)) & 0xFFFFu) ^ 0x8000u;
                const uint32_t hi = (c << 16) | zz;
                const int64_t col = cb + q;
                uint64_t key = 0;
                if (live && hi >= (uint32_t)(thr >> 40) && col >= c0 && col < c1)
                    key = ((uint64_t)hi << 40) | (0xFFFFFFFFFFull - (lbase + q));
                offer(key);
            }
        }
    }
    // rows are walked by wavefronts, columns by lanes: coalesced streaming
    for (int64_t row = wave; !kVec && row < bh; row += kFmThreads / 64) {
        const int64_t ly = lr0 + row;
        sync_thr();
        for (int64_t col0 = 0; col0 < bw; col0 += 64) {
            const int64_t col = col0 + lane;
            uint64_t key = 0;
            if (col < bw) {
                const int64_t lx = lc0 + col;
                const uint64_t local = (uint64_t)(row * bw + col);
                if (!kF32) {
                    const uint32_t c = ((const uint8_t *)keyp)[ly * ncols + lx];
                    const uint32_t zz = (uint16_t)z[ly * ld + lx] ^ 0x8000u;
                    key = ((uint64_t)c << 56) | ((uint64_t)zz << 40) | (0xFFFFFFFFFFull - local);
                } else {
                    const float f = ((const float *)keyp)[ly * kc + lx];
                    key = ((uint64_t)ord_f32(f) << 32) | (0xFFFFFFFFull - local);
                }
            }
            offer(key);
        }
    }
    // merge the wavefronts' lists: k rounds of a workgroup argmax, the lane
    // holding the winner drops it
    for (int rank = 0; rank < k; rank++) {
        const uint64_t mine = T;
        const uint64_t m = wave_max_u64(mine);
        if (lane == 0)
            wmax[wave] = m;
        __syncthreads();
        uint64_t best = wmax[0];
#pragma unroll
        for (int w = 1; w < kFmThreads / 64; w++)
            best = wmax[w] > best ? wmax[w] : best;
        // keys are unique: exactly one lane holds a non-zero maximum
        if (best != 0 && mine == best)
            T = 0;
        if (tid == 0) {
            int64_t out = -1;
            if (best != 0) {
                uint64_t local = kF32 ? (0xFFFFFFFFull - (best & 0xFFFFFFFFull))
                                      : (0xFFFFFFFFFFull - (best & 0xFFFFFFFFFFull));
                int64_t ly = lr0 + (int64_t)(local / (uint64_t)bw);
                int64_t lx = lc0 + (int64_t)(local % (uint64_t)bw);
                if (kF32) {
                    // the cell stands for its highest post (elevation desc,
                    // index asc)
                    int bz = -32769;
                    for (int64_t y = ly * stride; y < (ly + 1) * stride && y < nrows; y++)
                        for (int64_t x = lx * stride; x < (lx + 1) * stride && x < ncols; x++) {
                            const int v = z[y * ld + x];
                            if (v > bz) {
                                bz = v;
                                out = y * ncols + x;
                            }
                        }
                } else {
                    out = ly * ncols + lx;
                }
            }
            cand[blk * k + rank] = out;
        }
        __syncthreads();
    }
}

}  // namespace
}  // namespace siting

using namespace siting;

extern "C" int siting_findmax(const void *key, int32_t key_type, int32_t key_stride,
                              const int16_t *z, int64_t nrows, int64_t ncols, int64_t ld,
                              int32_t grid_r, int32_t grid_c, int32_t k, int64_t *cand,
                              void *stream)
{
    clear_error();
    SITING_REQUIRE(key != nullptr && cand != nullptr, "siting_findmax: NULL key or output");
    SITING_REQUIRE(key_type == SITING_KEY_U8 || key_type == SITING_KEY_F32,
                   "siting_findmax: unknown key_type %d", key_type);
    SITING_REQUIRE(z != nullptr, "siting_findmax: NULL terrain");
    SITING_REQUIRE(nrows >= 1 && ncols >= 1, "siting_findmax: empty terrain");
    SITING_REQUIRE(ld >= ncols, "siting_findmax: ld < ncols");
    SITING_REQUIRE(key_stride >= 1, "siting_findmax: key_stride must be >= 1");
    SITING_REQUIRE(key_type == SITING_KEY_F32 || key_stride == 1,
                   "siting_findmax: u8 keys need key_stride 1");
    SITING_REQUIRE(grid_r >= 1 && grid_r <= nrows && grid_c >= 1 && grid_c <= ncols,
                   "siting_findmax: grid %dx%d does not fit the %lldx%lld terrain", grid_r,
                   grid_c, (long long)nrows, (long long)ncols);
    SITING_REQUIRE(k >= 1, "siting_findmax: k must be >= 1");
    if (k > kFmMaxK) {
        set_error("siting_findmax: k %d above the supported %d", k, kFmMaxK);
        return SITING_E_UNSUPPORTED;
    }
    int64_t blocks = (int64_t)grid_r * grid_c;
    int64_t max_block = ((nrows + grid_r - 1) / grid_r) * ((ncols + grid_c - 1) / grid_c);
    if (blocks > INT32_MAX || (key_type == SITING_KEY_U8 && max_block >= (1ll << 40)) ||
        (key_type == SITING_KEY_F32 && max_block >= (1ll << 32))) {
        set_error("siting_findmax: blocks too large or too many");
        return SITING_E_UNSUPPORTED;
    }
    hipStream_t s = as_stream(stream);
    dim3 g((unsigned)blocks), b(kFmThreads);
    // 16-byte streaming when key rows (ncols bytes) and terrain rows (2*ld
    // bytes) start 16-byte aligned and a block's chunk count fits 32 bits
    const int64_t max_rows = (nrows + grid_r - 1) / grid_r + 1;
    const int64_t max_chunks = ((ncols + grid_c - 1) / grid_c + 32) / 16;
    const bool vec = key_type == SITING_KEY_U8 && ncols % 16 == 0 && ld % 8 == 0 &&
                     (uintptr_t)key % 16 == 0 && (uintptr_t)z % 16 == 0 &&
                     max_rows * max_chunks < ((int64_t)1 << 31);
    if (vec)
        hipLaunchKernelGGL((findmax_kernel<false, true>), g, b, 0, s, key, key_stride, z, nrows,
                           ncols, ld, grid_r, grid_c, k, cand);
    else if (key_type == SITING_KEY_U8)
        hipLaunchKernelGGL((findmax_kernel<false, false>), g, b, 0, s, key, key_stride, z, nrows,
                           ncols, ld, grid_r, grid_c, k, cand);
    else
        hipLaunchKernelGGL((findmax_kernel<true, false>), g, b, 0, s, key, key_stride, z, nrows,
                           ncols, ld, grid_r, grid_c, k, cand);
    return check_launch("findmax_kernel");
}
