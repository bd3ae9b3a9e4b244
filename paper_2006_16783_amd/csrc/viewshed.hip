// VIEWSHED: batched ray-sweep viewsheds in one persistent launch (stage
// Viewshed: walk around the ROI circle, run a line of sight to each point and
// walk along it updating a horizon; bitmaps in 64-bit words).
//
// Design (gfx950):
//  * Persistent workgroups pop observers from an atomic queue (the caller's
//    order, normally longest ROI first), so uneven ROIs balance themselves.
//  * The observer's window bitmap lives in LDS (rows x words, a row pitch of
//    an odd number of dwords so column-wise marks hit distinct banks) and is
//    written to HBM once, coalesced, in the global word alignment.
//  * The window is swept one half at a time (upper: quadrants 0 and 1, lower:
//    2 and 3).  A quadrant's rays read only posts inside it, so a workgroup
//    stages a half-window ((R+1) x (2R+1) int16) in LDS, half the window's LDS,
//    and sweeps both quadrants' rays together (about 4R rays, so the last
//    wavefront of a pass is rarely nearly empty).  Observers above the
//    schedule's stage_rmax read the terrain from global memory (L2 / Infinity
//    Cache) instead.
//  * Quadrant mode: when even the window bitmap exceeds LDS (ROI above 543),
//    every observer of the launch is swept one quadrant at a time from global
//    memory, the quadrant's bitmap in LDS; its words go out at once, ORed
//    where an earlier quadrant wrote the same word (the observer's row and
//    the word holding its column).
//  * Global-bitmap mode: when a quadrant's bitmap exceeds LDS too (ROI above
//    1087), the workgroup clears the observer's output window in HBM and its
//    rays mark cells there with atomic ORs (served by L2), the terrain read
//    through the cache hierarchy; same rays and comparisons.
//  * One ray per lane; consecutive lanes take consecutive boundary cells, so
//    a wavefront's rays have similar lengths and similar LDS rows.
//  * Exact integer slopes.  The per-quadrant elevation range bounds every
//    product; when (|z-E|max + h_r) * R^2 < 2^31 (almost always) the comparisons
//    run on the full-rate 24-bit multiplier in int32, otherwise in int64.
#include <algorithm>
#include <type_traits>

#include "common.hpp"

namespace siting {
namespace {

__device__ __forceinline__ int wave_min_i32(int v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1)
        v = min(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ int wave_max_i32(int v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1)
        v = max(v, __shfl_xor(v, o, 64));
    return v;
}

// Geometry of one quadrant in its local frame (u along the quadrant's first
// axis, v along the second; u > 0, v >= 0).  Global offsets of local (u, v):
//   Q0: ( u,  v)   Q1: (-v,  u)   Q2: (-u, -v)   Q3: ( v, -u)
struct Quadrant {
    int eu, ev;     // extents of the clipped window along u and v
    int bu, bv;     // bitmap bit-position steps of u and v
    int gu, gv;     // global terrain element steps of u and v
};

__device__ __forceinline__ Quadrant make_quadrant(int qd, int ex_p, int ex_m, int ey_p,
                                                  int ey_m, int BP, int ld)
{
    // ex_p = xhi - x, ex_m = x - xlo, ey_p = yhi - y, ey_m = y - ylo
    Quadrant Q;
    switch (qd) {
    case 0: Q.eu = ex_p; Q.ev = ey_p; Q.bu = 1;   Q.bv = BP;  Q.gu = 1;   Q.gv = ld;  break;
    case 1: Q.eu = ey_p; Q.ev = ex_m; Q.bu = BP;  Q.bv = -1;  Q.gu = ld;  Q.gv = -1;  break;
    case 2: Q.eu = ex_m; Q.ev = ey_m; Q.bu = -1;  Q.bv = -BP; Q.gu = -1;  Q.gv = -ld; break;
    default: Q.eu = ey_m; Q.ev = ex_p; Q.bu = -BP; Q.bv = 1;  Q.gu = -ld; Q.gv = 1;   break;
    }
    return Q;
}

// Boundary cell of ray rho (0 <= rho < eu + ev) in the local frame: first the
// far side u = eu (v = 0..ev), then the far side v = ev (u = eu-1..1).
__device__ __forceinline__ void ray_target(const Quadrant &Q, int rho, int &du, int &dv)
{
    if (rho <= Q.ev) {
        du = Q.eu;
        dv = rho;
    } else {
        du = Q.eu - (rho - Q.ev);
        dv = Q.ev;
    }
}

// Terrain sources.  `at(off)` reads the post at element offset `off` from the
// observer (LDS quadrant in the local frame, or the global terrain).
struct LdsSrc {
    const int16_t *p;
    __device__ __forceinline__ int at(int off) const { return p[off]; }
};
struct GlobalSrc {
    const int16_t *p;
    __device__ __forceinline__ int at(int off) const { return p[off]; }
};

// Sweep one ray to local boundary cell (du, dv).
//  zs_u, zs_v : terrain element steps of u and v in `src`
//  bm         : LDS bitmap (dwords); P0 the observer's bit position
// kGuardZ1: read the second post only when r > 0 (needed for global reads,
// where the padding post may lie outside the terrain).
template <bool kNarrow, bool kGuardZ1, class Src>
__device__ __forceinline__ void sweep(const Src &src, int zs_u, int zs_v, uint32_t *bm, int P0,
                                      int bu, int bv, int du, int dv, int R2, int E, int h_r)
{
    bool umaj = du >= dv;
    int n = umaj ? du : dv, mn = umaj ? dv : du;
    int zs_maj = umaj ? zs_u : zs_v, zs_min = umaj ? zs_v : zs_u;
    int bs_maj = umaj ? bu : bv, bs_min = umaj ? bv : bu;
    using W = typename std::conditional<kNarrow, int, long long>::type;
    int En = E * n;
    W hrn = (W)h_r * n;
    // step 1 (no horizon yet)
    int r = mn, q = 0;
    if (r >= n) {
        r -= n;
        q = 1;
    }
    int up = 2 * r >= n;
    int m = q + up;
    if (1 + m * m > R2)
        return;
    int zi = zs_maj + q * zs_min;
    int bq = P0 + bs_maj + q * bs_min;
    int z0 = src.at(zi);
    int z1 = (!kGuardZ1 || r) ? src.at(zi + zs_min) : 0;
    int S = __mul24(z0, n) + __mul24(z1 - z0, r);
    int T = S - En;
    {
        int bp = bq + (up ? bs_min : 0);
        atomicOr(&bm[bp >> 5], 1u << (bp & 31));
    }
    // horizon (hN, hJ): slope hN / hJ; B = hN * k for the current k
    W hN = T, hJ = 1, hrnJ = hrn, B = T;
    int k2 = 1;
    for (int k = 2; k <= n; k++) {
        r += mn;
        zi += zs_maj;
        bq += bs_maj;
        k2 += 2 * k - 1;
        if (r >= n) {
            r -= n;
            zi += zs_min;
            bq += bs_min;
            q++;
        }
        up = 2 * r >= n;
        m = q + up;
        if (k2 + __mul24(m, m) > R2)
            break;
        z0 = src.at(zi);
        z1 = (!kGuardZ1 || r) ? src.at(zi + zs_min) : 0;
        S = __mul24(z0, n) + __mul24(z1 - z0, r);
        T = S - En;
        B += hN;
        W PT, PV;
        if (kNarrow) {
            PT = __mul24((int)T, (int)hJ);
        } else {
            PT = (W)T * hJ;
        }
        PV = PT + hrnJ;
        if (PV >= B) {
            int bp = bq + (up ? bs_min : 0);
            atomicOr(&bm[bp >> 5], 1u << (bp & 31));
        }
        if (PT > B) {
            hN = T;
            hJ = k;
            if (kNarrow) {
                hrnJ = __mul24((int)hrn, k);
                B = __mul24(T, k);
            } else {
                hrnJ = hrn * k;
                B = (W)T * k;
            }
        }
    }
}

// One wavefront per ray (schedule ray_per_wave): the ray's samples are taken
// 64 at a time, sample k = 64c + lane + 1 on lane `lane` of chunk c, all with
// the same comparisons as sweep().  The horizon before sample k is the
// largest terrain slope T_j / j over j < k; the wavefront gets it as an
// exact prefix maximum of the rational slopes across lanes (DPP scan,
// cross-multiplied in int64; k == 0 marks "no sample"), shifted by one lane
// and combined with the maximum carried from earlier chunks.  Each lane
// advances its crossing (q, r) by 64 samples per chunk without division.
template <int kCtrl, int kRowMask>
__device__ __forceinline__ int dpp32(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, kCtrl, kRowMask, 0xF, false);
}
template <int kCtrl, int kRowMask>
__device__ __forceinline__ void scan_step(long long &T, int &k)
{
    const int lo = dpp32<kCtrl, kRowMask>((int)(uint32_t)(unsigned long long)T);
    const int hi = dpp32<kCtrl, kRowMask>((int)(uint32_t)((unsigned long long)T >> 32));
    const long long oT = (long long)(((unsigned long long)(uint32_t)hi << 32) | (uint32_t)lo);
    const int ok = dpp32<kCtrl, kRowMask>(k);
    if (ok != 0 && (k == 0 || oT * k > T * ok)) {
        T = oT;
        k = ok;
    }
}

template <bool kGuardZ1, class Src>
__device__ __forceinline__ void sweep_wave(const Src &src, int zs_u, int zs_v, uint32_t *bm,
                                           int P0, int bu, int bv, int du, int dv, int R2, int E,
                                           int h_r, int lane)
{
    const bool umaj = du >= dv;
    const int n = umaj ? du : dv, mn = umaj ? dv : du;
    const int zs_maj = umaj ? zs_u : zs_v, zs_min = umaj ? zs_v : zs_u;
    const int bs_maj = umaj ? bu : bv, bs_min = umaj ? bv : bu;
    const long long En = (long long)E * n, hrn = (long long)h_r * n;
    // crossing of sample k = lane + 1, and the advance of 64 samples
    int k = lane + 1;
    int q = (int)((uint32_t)(k * mn) / (uint32_t)n);
    int r = k * mn - q * n;
    const int dq = (int)((uint32_t)(64 * mn) / (uint32_t)n), dr = 64 * mn - dq * n;
    long long cT = 0;  // horizon carried from earlier chunks (ck == 0: none yet)
    int ck = 0;
    for (;;) {
        const int up = 2 * r >= n ? 1 : 0;
        const int m = q + up;
        const bool inside = k <= n && k * k + m * m <= R2;
        // the marked cells leave the disk for good: done when the chunk's
        // first sample is outside
        if (!(__ballot(inside) & 1ull))
            break;
        long long T = 0;
        if (inside) {
            const int zi = k * zs_maj + q * zs_min;
            const int z0 = src.at(zi);
            const int z1 = (!kGuardZ1 || r) ? src.at(zi + zs_min) : 0;
            T = (long long)z0 * (n - r) + (long long)z1 * r - En;
        }
        // inclusive prefix maximum of the slopes T / k over the chunk
        long long sT = T;
        int sk = inside ? k : 0;
        scan_step<0x111, 0xF>(sT, sk);
        scan_step<0x112, 0xF>(sT, sk);
        scan_step<0x114, 0xF>(sT, sk);
        scan_step<0x118, 0xF>(sT, sk);
        scan_step<0x142, 0xA>(sT, sk);
        scan_step<0x143, 0xC>(sT, sk);
        // exclusive: the previous lane's, then the carried horizon
        long long eT = (long long)(((unsigned long long)(uint32_t)__shfl_up(
                                        (int)(uint32_t)((unsigned long long)sT >> 32), 1, 64)
                                    << 32) |
                                   (uint32_t)__shfl_up((int)(uint32_t)(unsigned long long)sT, 1, 64));
        int ek = __shfl_up(sk, 1, 64);
        if (lane == 0) {
            eT = 0;
            ek = 0;
        }
        if (ck != 0 && (ek == 0 || cT * ek > eT * ck)) {
            eT = cT;
            ek = ck;
        }
        // the first sample of the ray has no horizon and is visible
        if (inside && (ek == 0 || (T + hrn) * ek >= eT * k)) {
            const int bp = P0 + k * bs_maj + m * bs_min;
            atomicOr(&bm[bp >> 5], 1u << (bp & 31));
        }
        // carry the chunk's maximum (lane 63 holds the inclusive maximum)
        const int tk = __builtin_amdgcn_readlane(sk, 63);
        const long long tT = (long long)(((unsigned long long)(uint32_t)__builtin_amdgcn_readlane(
                                              (int)(uint32_t)((unsigned long long)sT >> 32), 63)
                                          << 32) |
                                         (uint32_t)__builtin_amdgcn_readlane(
                                             (int)(uint32_t)(unsigned long long)sT, 63));
        if (tk != 0 && (ck == 0 || tT * ck > cT * tk)) {
            cT = tT;
            ck = tk;
        }
        k += 64;
        q += dq;
        r += dr;
        if (r >= n) {
            r -= n;
            q++;
        }
    }
}

// 24-bit signed multiply-add (full rate): a * b + c with |a|, |b| < 2^23.
__device__ __forceinline__ int mad_i24(int a, int b, int c)
{
    int r;
    asm("v_mad_i32_i24 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

// 24-bit signed multiply (full rate): a * b with |a|, |b| < 2^23.
__device__ __forceinline__ int mul_i24(int a, int b)
{
    int r;
    asm("v_mul_i32_i24 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

typedef const int16_t __attribute__((address_space(3))) lds_i16;
__device__ __forceinline__ int lds_read_i16(int addr)
{
    return *reinterpret_cast<lds_i16 *>((uintptr_t)(uint32_t)addr);
}

// The common case of sweep(): terrain staged in LDS, narrow arithmetic.  The
// same steps and comparisons in a cheaper form:
//  * the minor remainder is kept as e = r - n in [-n, -1], so that a wrap is
//    the carry of one add, and the interpolated terrain is
//    n*z(t) = z1*n + (z1 - z0)*e;
//  * the marked cell rounds up when 2r >= n, i.e. e >= -floor(n/2);
//  * up to a bound ks (computed per ray) every marked cell lies inside the
//    disk (k^2 + (q+1)^2 <= R^2), so those steps skip the disk test;
//  * the receiver's line is tested as T*J + h_r*n*J >= hN*k with one
//    multiply-add (h_r*n < 2^23 in narrow mode);
//  * post offsets are LDS byte addresses (zq_addr: the observer's post;
//    zs_u, zs_v: the byte steps of local u and v in the staged quadrant);
//    the post's address and the marked cell's bit position advance together
//    as one 64-bit value (bit position << 32 | address: both are
//    non-negative, so one 64-bit add of the packed signed steps is exact).
__device__ __forceinline__ void sweep_lds_narrow(int zq_addr, int zs_u, int zs_v, uint32_t *bm,
                                                 int P0, int bu, int bv, int du, int dv, int R2,
                                                 int E, int h_r)
{
    const bool umaj = du >= dv;
    const int n = umaj ? du : dv, mn = umaj ? dv : du;
    const int zs_maj = umaj ? zs_u : zs_v, zs_min = umaj ? zs_v : zs_u;
    const int bs_maj = umaj ? bu : bv, bs_min = umaj ? bv : bu;
    const int nEn = -E * n;
    const int hrn = h_r * n;
    const int nhalf = -(n >> 1);
    // step 1 (no horizon yet)
    int e = mn - n, q = 0;
    if (e >= 0) {  // the diagonal: mn == n
        e -= n;
        q = 1;
    }
    {
        const int m = q + (e >= nhalf ? 1 : 0);
        if (1 + m * m > R2)
            return;
    }
    int zi = zq_addr + zs_maj + q * zs_min;
    int bq = P0 + bs_maj + q * bs_min;
    int T;
    {
        const int z0 = lds_read_i16(zi), z1 = lds_read_i16(zi + zs_min);
        T = mad_i24(z1 - z0, e, mad_i24(z1, n, nEn));
        const int bp = bq + (e >= nhalf ? bs_min : 0);
        atomicOr(&bm[bp >> 5], 1u << (bp & 31));
    }
    int hN = T, hJ = 1, B = T;
    // ks: the last step whose marked cell is surely inside the disk, from
    // k^2 + (k*mn/n + 1)^2 <= R^2, then checked exactly
    int ks;
    {
        const float a = (float)mn / (float)n, c = 1.0f + a * a;
        const float root = (-a + sqrtf(a * a + c * (float)(R2 - 1))) / c;
        ks = (int)root;
        ks = ks < 1 ? 1 : ks > n ? n : ks;
        // (every product < 2^31: ks, mn <= n <= R <= 16383)
        while (ks > 1) {
            const int qq = (int)((uint32_t)(ks * mn) / (uint32_t)n) + 1;
            if (ks * ks + qq * qq <= R2)
                break;
            ks--;
        }
    }
    uint32_t eu = (uint32_t)e;
    uint64_t pos = ((uint64_t)(uint32_t)bq << 32) | (uint32_t)zi;
    const uint64_t d0 = (uint64_t)(((int64_t)bs_maj << 32) + zs_maj);
    const uint64_t d1 = (uint64_t)(((int64_t)(bs_maj + bs_min) << 32) + (zs_maj + zs_min));
    int k = 2;
    for (; k <= ks; k++) {
        uint32_t e1;
        const bool w = __builtin_add_overflow(eu, (uint32_t)mn, &e1);
        eu = w ? e1 - (uint32_t)n : e1;
        pos += w ? d1 : d0;
        zi = (int)(uint32_t)pos;
        bq = (int)(pos >> 32);
        const int ee = (int)eu;
        const int z0 = lds_read_i16(zi), z1 = lds_read_i16(zi + zs_min);
        const int Tk = mad_i24(z1 - z0, ee, mad_i24(z1, n, nEn));
        B += hN;
        const int PT = __mul24(Tk, hJ);
        const int PV = mad_i24(hrn, hJ, PT);
        const int bp = bq + (ee >= nhalf ? bs_min : 0);
        if (PV >= B)
            atomicOr(&bm[bp >> 5], 1u << (bp & 31));
        if (PT > B) {
            hN = Tk;
            hJ = k;
            B = mul_i24(Tk, k);
        }
    }
    if (k > n)
        return;
    // the remaining steps test the disk: q from the remainder, k^2 tracked
    q = (int)((uint32_t)((k - 1) * mn) / (uint32_t)n);
    int k2 = (k - 1) * (k - 1);
    for (; k <= n; k++) {
        uint32_t e1;
        const bool w = __builtin_add_overflow(eu, (uint32_t)mn, &e1);
        eu = w ? e1 - (uint32_t)n : e1;
        pos += w ? d1 : d0;
        zi = (int)(uint32_t)pos;
        bq = (int)(pos >> 32);
        q += w ? 1 : 0;
        k2 += 2 * k - 1;
        const int ee = (int)eu;
        const int up = ee >= nhalf ? 1 : 0;
        const int m = q + up;
        if (k2 + __mul24(m, m) > R2)
            break;
        const int z0 = lds_read_i16(zi), z1 = lds_read_i16(zi + zs_min);
        const int Tk = mad_i24(z1 - z0, ee, mad_i24(z1, n, nEn));
        B += hN;
        const int PT = __mul24(Tk, hJ);
        const int PV = mad_i24(hrn, hJ, PT);
        const int bp = bq + (up ? bs_min : 0);
        if (PV >= B)
            atomicOr(&bm[bp >> 5], 1u << (bp & 31));
        if (PT > B) {
            hN = Tk;
            hJ = k;
            B = mul_i24(Tk, k);
        }
    }
}

// LDS layout helpers (bytes), shared by host sizing and the kernel.
__host__ __device__ __forceinline__ int bm_pitch_dw(int rmax)
{
    int nw = ((2 * rmax) >> 6) + 2;  // max 64-bit words a window row spans
    return 2 * nw + 1;               // odd dword pitch
}
__host__ __device__ __forceinline__ int bm_bytes(int rmax)
{
    return (2 * rmax + 1) * bm_pitch_dw(rmax) * 4;
}
// Quadrant mode (windows too large for LDS): one quadrant's bitmap at a time,
// (rmax+1) rows of at most (rmax>>6)+2 words, odd dword pitch.
__host__ __device__ __forceinline__ int bmq_pitch_dw(int rmax)
{
    return 2 * ((rmax >> 6) + 2) + 1;
}
__host__ __device__ __forceinline__ int bmq_bytes(int rmax)
{
    // plus the count sink's row and column masks (2R+1 bits each)
    return (rmax + 1) * bmq_pitch_dw(rmax) * 4 + 2 * ((2 * rmax + 1 + 31) >> 5) * 4;
}
// A staged half-window (at most rmax+1 rows of 2*rmax+1 posts) keeps the
// terrain's orientation; its rows start at an even terrain column, so a row
// spans at most 2*rmax+2 posts, and an odd dword pitch puts a column's posts in
// distinct banks.  A ray whose line meets a post exactly still reads the next
// post along the minor axis (with weight zero), which can lie one row past the
// box: one spare row keeps that read inside the allocation.
__host__ __device__ __forceinline__ int zq_pitch_dw(int rmax)
{
    return (rmax + 1) | 1;
}
__host__ __device__ __forceinline__ int zq_bytes(int rmax)
{
    return rmax > 0 ? (rmax + 2) * zq_pitch_dw(rmax) * 4 : 0;
}

__global__ void viewshed_queue_reset(uint32_t *queue) { queue[0] = 0; }

__device__ __forceinline__ int isqrt_floor(int v)
{
    int s = (int)sqrtf((float)v);
    while (s > 0 && s * s > v)
        s--;
    while ((s + 1) * (s + 1) <= v)
        s++;
    return s;
}

// One instantiation per mode and ray schedule, so that the common path (mode
// 0, a lane per ray) carries neither the other modes' code nor the
// wavefront-per-ray sweep's registers.
template <int kMode, bool kRayWave>
__global__ void viewshed_kernel(const int16_t *__restrict__ z, int64_t nrows, int64_t ncols,
                                int64_t ld, const siting_observer *__restrict__ obs, int64_t n,
                                const int64_t *__restrict__ offsets,
                                const int32_t *__restrict__ order, int sink,
                                uint64_t *__restrict__ bitmaps, uint32_t *__restrict__ visible,
                                uint32_t *__restrict__ cells, uint32_t *queue, int rmax,
                                int stage_rmax, int dma)
{
    // mode 0: window bitmap in LDS; 1: quadrant mode; 2: global-bitmap mode
    constexpr int mode = kMode;
    constexpr bool ray_wave = kRayWave;
    constexpr bool quad = mode == 1;
    extern __shared__ uint32_t lds[];
    __shared__ int64_t s_task;
    __shared__ int s_red[2 * 16];
    __shared__ uint32_t s_sum[2 * 16];
    const int tid = threadIdx.x, nthreads = blockDim.x;
    const int wave = tid >> 6, lane = tid & 63, nwaves = nthreads >> 6;
    uint32_t *bm = lds;
    int16_t *zq = reinterpret_cast<int16_t *>(lds + bm_bytes(rmax) / 4);
    const int zpd = zq_pitch_dw(stage_rmax);  // staged row pitch (dwords)
    // LDS byte address of the staged box
    const int zq_addr =
        (int)(uint32_t)(uintptr_t)(const __attribute__((address_space(3))) int16_t *)zq;
    const int BPdw = bm_pitch_dw(rmax);
    const int BP = BPdw * 32;

    for (;;) {
        if (tid == 0)
            s_task = atomicAdd(queue, 1u);
        __syncthreads();
        int64_t task = s_task;
        if (task >= n)
            break;
        int64_t i = order ? order[task] : task;
        siting_observer o = obs[i];
        // records the host did not validate: never touch memory for them
        if (o.roi < 1 || o.roi > rmax || o.x < 0 || o.x >= ncols || o.y < 0 || o.y >= nrows ||
            o.h_t < 0 || o.h_t > kMaxHeight || o.h_r < 0 || o.h_r > kMaxHeight) {
            if (sink == SITING_SINK_COUNT && tid == 0) {
                visible[i] = 0;
                cells[i] = 0;
            }
            __syncthreads();
            continue;
        }
        const int R = o.roi;
        const int64_t x = o.x, y = o.y;
        const int64_t xlo = x - R < 0 ? 0 : x - R, xhi = x + R > ncols - 1 ? ncols - 1 : x + R;
        const int64_t ylo = y - R < 0 ? 0 : y - R, yhi = y + R > nrows - 1 ? nrows - 1 : y + R;
        const int64_t w0 = xlo >> 6;
        const int nw = (int)((xhi >> 6) - w0 + 1);
        const int rows = (int)(yhi - ylo + 1);
        const int ex_p = (int)(xhi - x), ex_m = (int)(x - xlo);
        const int ey_p = (int)(yhi - y), ey_m = (int)(y - ylo);
        const int P0 = (int)(y - ylo) * BP + (int)(x - (w0 << 6));
        const int R2 = R * R;
        const int16_t *zo = z + y * ld + x;
        const int E = (int)zo[0] + o.h_t;

        if (mode == 2) {
            // the window bitmap in HBM (with the count sink, the caller's
            // bitmaps serve as scratch): cleared, then marked by every ray of
            // the four quadrants with atomic ORs on its dwords (bit b of the
            // row-major bit array is bit b & 31 of dword b >> 5)
            uint64_t *out = bitmaps + offsets[i];
            const int words = rows * nw;
            for (int e = tid; e < words; e += nthreads)
                out[e] = 0;
            __threadfence();
            __syncthreads();
            uint32_t *gbm = reinterpret_cast<uint32_t *>(out);
            const int GP = nw * 64;  // bits per window row (< 2^31 / rows)
            const int P0g = (int)(y - ylo) * GP + (int)(x - (w0 << 6));
            if (tid == 0)
                atomicOr(&gbm[P0g >> 5], 1u << (P0g & 31));
            const int n0 = ex_p >= 1 ? ex_p + ey_p : 0;
            const int n1 = n0 + (ey_p >= 1 ? ey_p + ex_m : 0);
            const int n2 = n1 + (ex_m >= 1 ? ex_m + ey_m : 0);
            const int n3 = n2 + (ey_m >= 1 ? ey_m + ex_p : 0);
            GlobalSrc src{zo};
            const int r0 = ray_wave ? wave : tid, rs = ray_wave ? nwaves : nthreads;
            for (int rho = r0; rho < n3; rho += rs) {
                const int qd = rho < n0 ? 0 : rho < n1 ? 1 : rho < n2 ? 2 : 3;
                const int base = qd == 0 ? 0 : qd == 1 ? n0 : qd == 2 ? n1 : n2;
                const Quadrant Q = make_quadrant(qd, ex_p, ex_m, ey_p, ey_m, GP, (int)ld);
                int du, dv;
                ray_target(Q, rho - base, du, dv);
                if (ray_wave)
                    sweep_wave<true>(src, Q.gu, Q.gv, gbm, P0g, Q.bu, Q.bv, du, dv, R2, E, o.h_r,
                                     lane);
                else
                    sweep<false, true>(src, Q.gu, Q.gv, gbm, P0g, Q.bu, Q.bv, du, dv, R2, E,
                                       o.h_r);
            }
            __threadfence();
            __syncthreads();
            if (sink == SITING_SINK_COUNT) {
                // visible cells: the window's set bits; disk cells row by row
                uint32_t vis = 0, cnt = 0;
                for (int e = tid; e < words; e += nthreads)
                    vis += (uint32_t)__popcll(out[e]);
                for (int row = tid; row < rows; row += nthreads) {
                    const int dy = (int)(ylo + row - y);
                    const int hw = isqrt_floor(R2 - dy * dy);
                    const int64_t a = x - hw < xlo ? xlo : x - hw;
                    const int64_t b = x + hw > xhi ? xhi : x + hw;
                    if (b >= a)
                        cnt += (uint32_t)(b - a + 1);
                }
                vis = wave_sum_u32(vis);
                cnt = wave_sum_u32(cnt);
                if (lane == 0) {
                    s_sum[wave] = vis;
                    s_sum[16 + wave] = cnt;
                }
                __syncthreads();
                if (tid == 0) {
                    uint32_t tv = 0, tc = 0;
                    for (int w = 0; w < nwaves; w++) {
                        tv += s_sum[w];
                        tc += s_sum[16 + w];
                    }
                    visible[i] = tv;
                    cells[i] = tc;
                }
                __syncthreads();
            }
            continue;
        }

        if (quad) {
            // one quadrant at a time in LDS, terrain from global memory; each
            // quadrant's words go out at once, ORed where an earlier quadrant
            // wrote the same word (the observer's row and the word holding
            // its column), so the window is written exactly once over
            const int QPdw = bmq_pitch_dw(rmax), QP = QPdw * 32;
            const int64_t xw = x >> 6;
            uint32_t vis = 0;
            GlobalSrc src{zo};
            // count sink: masks of the visible cells on the observer's row
            // (bit c - xlo) and column (bit r - ylo), after the bitmap
            const int axdw = (2 * rmax + 1 + 31) >> 5;
            uint32_t *axr = bm + (rmax + 1) * QPdw, *axc = axr + axdw;
            if (sink == SITING_SINK_COUNT)
                for (int e = tid; e < 2 * axdw; e += nthreads)
                    axr[e] = 0;
            for (int qd = 0; qd < 4; qd++) {
                const int64_t row0 = qd < 2 ? y : ylo;
                const int nrq = qd < 2 ? ey_p + 1 : ey_m + 1;
                const int64_t c0 = (qd == 0 || qd == 3) ? x : xlo;
                const int64_t c1 = (qd == 0 || qd == 3) ? xhi : x;
                const int64_t word0 = c0 >> 6;
                const int nwq = (int)((c1 >> 6) - word0 + 1);
                const int P0q = (int)(y - row0) * QP + (int)(x - (word0 << 6));
                for (int e = tid; e < nrq * QPdw; e += nthreads)
                    bm[e] = 0;
                __syncthreads();
                if (tid == 0)
                    atomicOr(&bm[P0q >> 5], 1u << (P0q & 31));
                const Quadrant Q = make_quadrant(qd, ex_p, ex_m, ey_p, ey_m, QP, (int)ld);
                const int nrays = Q.eu >= 1 ? Q.eu + Q.ev : 0;
                const int q0 = ray_wave ? wave : tid, qs = ray_wave ? nwaves : nthreads;
                for (int rho = q0; rho < nrays; rho += qs) {
                    int du, dv;
                    ray_target(Q, rho, du, dv);
                    if (ray_wave)
                        sweep_wave<true>(src, Q.gu, Q.gv, bm, P0q, Q.bu, Q.bv, du, dv, R2, E,
                                         o.h_r, lane);
                    else
                        sweep<false, true>(src, Q.gu, Q.gv, bm, P0q, Q.bu, Q.bv, du, dv, R2, E,
                                           o.h_r);
                }
                __syncthreads();
                if (sink == SITING_SINK_BITMAP) {
                    uint64_t *out = bitmaps + offsets[i];
                    for (int e = tid; e < nrq * nwq; e += nthreads) {
                        const int r = e / nwq, w = e - r * nwq;
                        const int64_t grow = row0 + r, gw = word0 + w;
                        const uint32_t *q = bm + r * QPdw + 2 * w;
                        const uint64_t val = (uint64_t)q[0] | ((uint64_t)q[1] << 32);
                        uint64_t *dst = out + (grow - ylo) * nw + (gw - w0);
                        const bool shared = (qd == 1 && gw == xw) || (qd == 2 && grow == y) ||
                                            (qd == 3 && (grow == y || gw == xw));
                        if (shared)
                            *dst |= val;
                        else
                            *dst = val;
                    }
                } else {
                    // count each cell once: the observer's row and column,
                    // which two quadrants share, are ORed into the axis masks
                    // and cleared here; the rest is this quadrant's alone
                    const int xb = (int)(x - (word0 << 6)), ry = (int)(y - row0);
                    for (int64_t c = c0 + tid; c <= c1; c += nthreads) {
                        const int b = ry * QP + (int)(c - (word0 << 6));
                        if ((bm[b >> 5] >> (b & 31)) & 1u)
                            atomicOr(&axr[(c - xlo) >> 5], 1u << ((c - xlo) & 31));
                    }
                    for (int r = tid; r < nrq; r += nthreads) {
                        const int b = r * QP + xb;
                        const int64_t gr = row0 + r - ylo;
                        if ((bm[b >> 5] >> (b & 31)) & 1u)
                            atomicOr(&axc[gr >> 5], 1u << (gr & 31));
                    }
                    __syncthreads();
                    for (int r = tid; r < nrq; r += nthreads)
                        bm[r * QPdw + (xb >> 5)] &= ~(1u << (xb & 31));
                    __syncthreads();
                    for (int e = tid; e < QPdw; e += nthreads)
                        bm[ry * QPdw + e] = 0;
                    __syncthreads();
                    for (int e = tid; e < nrq * QPdw; e += nthreads)
                        vis += __popc(bm[e]);
                }
                __syncthreads();
            }
            if (sink == SITING_SINK_COUNT) {
                // the axes: row y from the row mask, column x (without the
                // observer's own cell, already in the row) from the column mask
                const int yb = (int)(y - ylo);
                for (int e = tid; e < axdw; e += nthreads) {
                    const uint32_t cm = e == (yb >> 5) ? axc[e] & ~(1u << (yb & 31)) : axc[e];
                    vis += __popc(axr[e]) + __popc(cm);
                }
                uint32_t cnt = 0;
                for (int row = tid; row < rows; row += nthreads) {
                    int dy = (int)(ylo + row - y);
                    int hw = isqrt_floor(R2 - dy * dy);
                    int64_t a = x - hw < xlo ? xlo : x - hw;
                    int64_t b = x + hw > xhi ? xhi : x + hw;
                    if (b >= a)
                        cnt += (uint32_t)(b - a + 1);
                }
                vis = wave_sum_u32(vis);
                cnt = wave_sum_u32(cnt);
                if (lane == 0) {
                    s_sum[wave] = vis;
                    s_sum[16 + wave] = cnt;
                }
                __syncthreads();
                if (tid == 0) {
                    uint32_t tv = 0, tc = 0;
                    for (int w = 0; w < nwaves; w++) {
                        tv += s_sum[w];
                        tc += s_sum[16 + w];
                    }
                    visible[i] = tv;
                    cells[i] = tc;
                }
            }
            __syncthreads();
            continue;
        }

        for (int e = tid; e < rows * BPdw; e += nthreads)
            bm[e] = 0;
        __syncthreads();
        if (tid == 0)
            atomicOr(&bm[P0 >> 5], 1u << (P0 & 31));

        if (R <= stage_rmax) {
            for (int half = 0; half < 2; half++) {
                // quadrants qa, qb = 0, 1 (rows y .. y+ey_p) or 2, 3 (rows
                // y-ey_m .. y); columns x-ex_m .. x+ex_p
                const int qa = 2 * half, qb = qa + 1;
                const Quadrant QA = make_quadrant(qa, ex_p, ex_m, ey_p, ey_m, BP, (int)ld);
                const Quadrant QB = make_quadrant(qb, ex_p, ex_m, ey_p, ey_m, BP, (int)ld);
                const int nA = QA.eu >= 1 ? QA.eu + QA.ev : 0;
                const int nB = QB.eu >= 1 ? QB.eu + QB.ev : 0;
                if (nA + nB == 0)
                    continue;
                const int64_t gx0 = x - ex_m, gx1 = x + ex_p;
                const int64_t gy0 = half ? y - ey_m : y, gy1 = half ? y : y + ey_p;
                // stage the half-window in the terrain's orientation, its rows
                // from the even column gxe
                int zmin = 32767, zmax = -32768;
                const int bw = (int)(gx1 - gx0 + 1), bh = (int)(gy1 - gy0 + 1);
                const int64_t gxe = gx0 & ~(int64_t)1;
                const int c0 = (int)(gx0 - gxe);
                if (dma) {
                    // each wavefront streams its rows straight into LDS
                    // (global_load_lds: lane i writes the dword at the LDS base
                    // + 4i), all of them in flight before one wait.  With ld and
                    // ncols even every dword lies inside its row.
                    const int ndw = (int)((gx1 - gxe) >> 1) + 1;
                    uint32_t *zd = reinterpret_cast<uint32_t *>(zq);
                    for (int r = wave; r < bh; r += nwaves) {
                        const uint32_t *srow =
                            reinterpret_cast<const uint32_t *>(z + (gy0 + r) * ld + gxe);
                        for (int k0 = 0; k0 < ndw; k0 += 64)
                            if (k0 + lane < ndw)
                                __builtin_amdgcn_global_load_lds(srow + k0 + lane,
                                                                 zd + r * zpd + k0, 4, 0, 0);
                    }
                    __builtin_amdgcn_s_waitcnt(0);
                    __syncthreads();
                    // elevation range (a post left of gx0 or right of gx1 is
                    // terrain too: it can only widen the range)
                    for (int r = wave; r < bh; r += nwaves)
                        for (int k = lane; k < ndw; k += 64) {
                            const uint32_t d = zd[r * zpd + k];
                            const int lo = (int)(int16_t)(d & 0xFFFFu), hi = (int)(int16_t)(d >> 16);
                            zmin = min(zmin, min(lo, hi));
                            zmax = max(zmax, max(lo, hi));
                        }
                } else {
                    // four rows per wavefront and two 64-post chunks per row
                    // in flight before the LDS writes
                    for (int row = wave; row < bh; row += 4 * nwaves) {
                        const int16_t *sp[4];
                        int rb[4];
                        bool rv[4];
#pragma unroll
                        for (int u = 0; u < 4; u++) {
                            const int r = row + u * nwaves;
                            rv[u] = r < bh;
                            sp[u] = z + (gy0 + (rv[u] ? r : 0)) * ld + gx0;
                            rb[u] = r * 2 * zpd + c0;
                        }
                        for (int cc = lane; cc < bw; cc += 128) {
                            int v[4][2];
#pragma unroll
                            for (int u = 0; u < 4; u++)
#pragma unroll
                                for (int h = 0; h < 2; h++) {
                                    const int col = cc + 64 * h;
                                    v[u][h] = rv[u] && col < bw ? (int)sp[u][col] : 0;
                                }
#pragma unroll
                            for (int u = 0; u < 4; u++)
#pragma unroll
                                for (int h = 0; h < 2; h++) {
                                    const int col = cc + 64 * h;
                                    if (rv[u] && col < bw) {
                                        zq[rb[u] + col] = (int16_t)v[u][h];
                                        zmin = min(zmin, v[u][h]);
                                        zmax = max(zmax, v[u][h]);
                                    }
                                }
                        }
                    }
                }
                zmin = wave_min_i32(zmin);
                zmax = wave_max_i32(zmax);
                if (lane == 0) {
                    s_red[wave] = zmin;
                    s_red[16 + wave] = zmax;
                }
                __syncthreads();
                int gmin = s_red[0], gmax = s_red[16];
                for (int w = 1; w < nwaves; w++) {
                    gmin = min(gmin, s_red[w]);
                    gmax = max(gmax, s_red[16 + w]);
                }
                long long D = max((long long)gmax - E, (long long)E - gmin) + o.h_r;
                bool narrow = D * R < (1ll << 23) && D * R * R < (1ll << 31);
                // the observer's post in the staged box, and the steps of each
                // quadrant's local u and v (elements; x is +1, y is +2*zpd):
                //   0: (u, v) = (x, y)   1: (y, -x)   2: (-x, -y)   3: (-y, x)
                const int zo_el = (int)(y - gy0) * 2 * zpd + (int)(x - gxe);
                const int sy = 2 * zpd;
                LdsSrc src{zq + zo_el};
                const int zo_addr = zq_addr + 2 * zo_el;
                // rays of the two quadrants alternate, and within a quadrant
                // threads take the boundary cells from both ends inwards: the
                // near-axis rays (longest) fill the first wavefronts, and the
                // last one gets near-diagonal rays, which leave the disk first
                const int m2 = 2 * min(nA, nB);
                for (int t = tid; t < nA + nB; t += nthreads) {
                    int qs, idx;
                    if (t < m2) {
                        qs = t & 1;
                        idx = t >> 1;
                    } else {
                        qs = nA > nB ? 0 : 1;
                        idx = t - m2 + (m2 >> 1);
                    }
                    const Quadrant &Q = qs ? QB : QA;
                    const int nq = qs ? nB : nA;
                    const int rho = (idx & 1) ? nq - 1 - (idx >> 1) : (idx >> 1);
                    const int su = half ? (qs ? -sy : -1) : (qs ? sy : 1);
                    const int sv = half ? (qs ? 1 : -sy) : (qs ? -1 : sy);
                    int du, dv;
                    ray_target(Q, rho, du, dv);
                    if (narrow)
                        sweep_lds_narrow(zo_addr, 2 * su, 2 * sv, bm, P0, Q.bu, Q.bv, du, dv, R2,
                                         E, o.h_r);
                    else
                        sweep<false, false>(src, su, sv, bm, P0, Q.bu, Q.bv, du, dv, R2, E, o.h_r);
                }
                __syncthreads();
            }
        } else {
            // global terrain reads; the four quadrants' rays in one pass
            int n0 = ex_p >= 1 ? ex_p + ey_p : 0;
            int n1 = n0 + (ey_p >= 1 ? ey_p + ex_m : 0);
            int n2 = n1 + (ex_m >= 1 ? ex_m + ey_m : 0);
            int n3 = n2 + (ey_m >= 1 ? ey_m + ex_p : 0);
            GlobalSrc src{zo};
            const int r0 = ray_wave ? wave : tid, rs = ray_wave ? nwaves : nthreads;
            for (int rho = r0; rho < n3; rho += rs) {
                int qd = rho < n0 ? 0 : rho < n1 ? 1 : rho < n2 ? 2 : 3;
                int base = qd == 0 ? 0 : qd == 1 ? n0 : qd == 2 ? n1 : n2;
                Quadrant Q = make_quadrant(qd, ex_p, ex_m, ey_p, ey_m, BP, (int)ld);
                int du, dv;
                ray_target(Q, rho - base, du, dv);
                if (ray_wave)
                    sweep_wave<true>(src, Q.gu, Q.gv, bm, P0, Q.bu, Q.bv, du, dv, R2, E, o.h_r,
                                     lane);
                else
                    sweep<false, true>(src, Q.gu, Q.gv, bm, P0, Q.bu, Q.bv, du, dv, R2, E, o.h_r);
            }
            __syncthreads();
        }

        if (sink == SITING_SINK_BITMAP) {
            uint64_t *out = bitmaps + offsets[i];
            const int words = rows * nw;
            for (int e = tid; e < words; e += nthreads) {
                int row = e / nw, w = e - row * nw;
                const uint32_t *src = bm + row * BPdw + 2 * w;
                out[e] = (uint64_t)src[0] | ((uint64_t)src[1] << 32);
            }
        } else {
            uint32_t vis = 0, cnt = 0;
            for (int e = tid; e < rows * BPdw; e += nthreads)
                vis += __popc(bm[e]);
            for (int row = tid; row < rows; row += nthreads) {
                int dy = (int)(ylo + row - y);
                int half = isqrt_floor(R2 - dy * dy);
                int64_t a = x - half < xlo ? xlo : x - half;
                int64_t b = x + half > xhi ? xhi : x + half;
                if (b >= a)
                    cnt += (uint32_t)(b - a + 1);
            }
            vis = wave_sum_u32(vis);
            cnt = wave_sum_u32(cnt);
            if (lane == 0) {
                s_sum[wave] = vis;
                s_sum[16 + wave] = cnt;
            }
            __syncthreads();
            if (tid == 0) {
                uint32_t tv = 0, tc = 0;
                for (int w = 0; w < nwaves; w++) {
                    tv += s_sum[w];
                    tc += s_sum[16 + w];
                }
                visible[i] = tv;
                cells[i] = tc;
            }
        }
        __syncthreads();
    }
}

}  // namespace

int viewshed_max_dynamic_lds()
{
    return kernel_max_dynamic_lds(reinterpret_cast<const void *>(&viewshed_kernel<0, false>));
}

// Windows whose bitmap exceeds LDS run in quadrant mode (terrain from global
// memory, staging off); windows whose quadrant bitmap exceeds it too, in
// global-bitmap mode.
int viewshed_mode(int rmax)
{
    if (bm_bytes(rmax) <= viewshed_max_dynamic_lds())
        return 0;
    return bmq_bytes(rmax) <= viewshed_max_dynamic_lds() ? 1 : 2;
}
bool quad_mode(int rmax) { return viewshed_mode(rmax) != 0; }

int lds_bytes_for(int rmax, int stage_rmax)
{
    const int mode = viewshed_mode(rmax);
    if (mode == 2)
        return 0;
    if (mode == 1)
        return bmq_bytes(rmax);
    return bm_bytes(rmax) + zq_bytes(std::min(stage_rmax, rmax));
}


int viewshed_launch(const int16_t *z, int64_t nrows, int64_t ncols, int64_t ld,
                    const siting_observer *obs, int64_t n, const int64_t *offsets,
                    const int32_t *order, int32_t rmax, const siting_schedule &sc, int32_t sink,
                    uint64_t *bitmaps, uint32_t *visible, uint32_t *cells, void *ws,
                    hipStream_t s)
{
    const int mode = viewshed_mode(rmax);
    if (mode == 2 && (bitmaps == nullptr || offsets == nullptr)) {
        set_error("siting_viewshed_batch: above rmax 1087 the windows are built in `bitmaps` "
                  "(with offsets), also for the count sink");
        return SITING_E_INVALID;
    }
    int stage = mode ? 0 : std::min(sc.stage_rmax, rmax);
    int lds = lds_bytes_for(rmax, stage);
    if (lds > viewshed_max_dynamic_lds()) {
        set_error("siting_viewshed_batch: schedule needs %d bytes of LDS (at most %d)", lds,
                  viewshed_max_dynamic_lds());
        return SITING_E_UNSUPPORTED;
    }
    int64_t grid = (int64_t)device_cus() * sc.groups_per_cu;
    if (grid > n)
        grid = n;
    uint32_t *queue = reinterpret_cast<uint32_t *>(ws);
    hipLaunchKernelGGL(viewshed_queue_reset, dim3(1), dim3(1), 0, s, queue);
    int rc = check_launch("viewshed_queue_reset");
    if (rc != SITING_OK)
        return rc;
    if (grid <= 0)
        return SITING_OK;
    // direct HBM-to-LDS staging needs dword-aligned rows that hold whole dwords
    const int dma = ld % 2 == 0 && ncols % 2 == 0 && reinterpret_cast<uintptr_t>(z) % 4 == 0;
    const bool rw = sc.ray_per_wave != 0;
    decltype(&viewshed_kernel<0, false>) k =
        mode == 0 ? (rw ? viewshed_kernel<0, true> : viewshed_kernel<0, false>)
        : mode == 1 ? (rw ? viewshed_kernel<1, true> : viewshed_kernel<1, false>)
                    : (rw ? viewshed_kernel<2, true> : viewshed_kernel<2, false>);
    hipLaunchKernelGGL(k, dim3((unsigned)grid), dim3(64 * sc.waves), (size_t)lds, s, z, nrows,
                       ncols, ld, obs, n, offsets, order, sink, bitmaps, visible, cells, queue,
                       rmax, stage, dma);
    return check_launch("viewshed_kernel");
}

int viewshed_default_schedule(int32_t rmax, siting_schedule *sc)
{
    const int budget = 160 * 1024;
    sc->ray_per_wave = 0;
    int lds_staged = lds_bytes_for(rmax, rmax);
    if (rmax <= 160 && lds_staged <= std::min(budget, viewshed_max_dynamic_lds())) {
        // a half-window has about 4R rays: enough wavefronts to sweep them in
        // one pass, plus one, at most 8
        sc->waves = std::max(2, std::min(8, (4 * rmax + 63) / 64 + 1));
        sc->stage_rmax = rmax;
        sc->groups_per_cu = std::max(1, std::min(8, budget / lds_staged));
    } else if (viewshed_mode(rmax) == 2) {
        // no LDS bitmap: two workgroups of 16 wavefronts per CU (8R rays
        // per observer)
        sc->stage_rmax = 0;
        sc->waves = 16;
        sc->groups_per_cu = 2;
    } else if (quad_mode(rmax)) {
        // one workgroup per CU holds a quadrant's bitmap; its 2R rays fill
        // 16 wavefronts about twice
        sc->stage_rmax = 0;
        sc->waves = 16;
        sc->groups_per_cu = 1;
    } else {
        // at least 16 wavefronts per CU: a workgroup whose bitmap takes the
        // CU's LDS alone gets 16 (1.5x faster than 8 at R = 500)
        sc->stage_rmax = 0;
        sc->groups_per_cu = std::max(1, std::min(8, budget / bm_bytes(rmax)));
        sc->waves = sc->groups_per_cu >= 2 ? 8 : 16;
    }
    return SITING_OK;
}

int viewshed_lds_bytes(int32_t rmax, int32_t stage_rmax) { return lds_bytes_for(rmax, stage_rmax); }

int validate_schedule(const siting_schedule &sc, const char *fn)
{
    SITING_REQUIRE(sc.waves >= 1 && sc.waves <= 16, "%s: schedule waves %d outside 1..16", fn,
                   sc.waves);
    SITING_REQUIRE(sc.groups_per_cu >= 1 && sc.groups_per_cu <= 16,
                   "%s: schedule groups_per_cu %d outside 1..16", fn, sc.groups_per_cu);
    SITING_REQUIRE(sc.stage_rmax >= 0 && sc.stage_rmax <= kMaxRoi,
                   "%s: schedule stage_rmax out of range", fn);
    SITING_REQUIRE(sc.ray_per_wave == 0 || sc.ray_per_wave == 1,
                   "%s: schedule ray_per_wave must be 0 or 1", fn);
    return SITING_OK;
}


}  // namespace siting

using namespace siting;

extern "C" size_t siting_viewshed_workspace_size(void) { return 256; }

extern "C" int siting_viewshed_default_schedule(int32_t rmax, siting_schedule *sched_host)
{
    clear_error();
    SITING_REQUIRE(sched_host != nullptr, "siting_viewshed_default_schedule: NULL output");
    SITING_REQUIRE(rmax >= 1 && rmax <= kMaxRoi, "siting_viewshed_default_schedule: bad rmax");
    return viewshed_default_schedule(rmax, sched_host);
}

extern "C" int siting_viewshed_batch(const int16_t *z, int64_t nrows, int64_t ncols, int64_t ld,
                                     const siting_observer *obs, int64_t n, const int64_t *offsets,
                                     const int32_t *order, int32_t rmax,
                                     const siting_schedule *sched_host, int32_t sink,
                                     uint64_t *bitmaps, uint32_t *visible, uint32_t *cells,
                                     void *ws, size_t ws_bytes, void *stream)
{
    clear_error();
    const char *fn = "siting_viewshed_batch";
    SITING_REQUIRE(n >= 0 && n <= INT32_MAX, "%s: n out of range", fn);
    SITING_REQUIRE(nrows >= 1 && ncols >= 1, "%s: empty terrain", fn);
    SITING_REQUIRE(ld >= ncols, "%s: ld < ncols", fn);
    SITING_REQUIRE(rmax >= 1 && rmax <= kMaxRoi, "%s: rmax %d outside 1..%d", fn, rmax, kMaxRoi);
    SITING_REQUIRE(sink == SITING_SINK_BITMAP || sink == SITING_SINK_COUNT, "%s: bad sink", fn);
    if (n == 0)
        return SITING_OK;
    SITING_REQUIRE(z != nullptr && obs != nullptr, "%s: NULL terrain or observers", fn);
    SITING_REQUIRE(sink != SITING_SINK_BITMAP || (bitmaps != nullptr && offsets != nullptr),
                   "%s: bitmap sink needs bitmaps and offsets", fn);
    SITING_REQUIRE(sink != SITING_SINK_COUNT || (visible != nullptr && cells != nullptr),
                   "%s: count sink needs visible and cells", fn);
    if (ws == nullptr || ws_bytes < siting_viewshed_workspace_size()) {
        set_error("%s: workspace of %zu bytes needed", fn, siting_viewshed_workspace_size());
        return SITING_E_WORKSPACE;
    }
    if ((int64_t)(rmax + 2) * ld >= ((int64_t)1 << 31)) {
        set_error("%s: rmax*ld too large for 32-bit offsets", fn);
        return SITING_E_UNSUPPORTED;
    }
    siting_schedule sc;
    if (sched_host) {
        sc = *sched_host;
        int rc = validate_schedule(sc, fn);
        if (rc != SITING_OK)
            return rc;
    } else {
        viewshed_default_schedule(rmax, &sc);
    }
    return viewshed_launch(z, nrows, ncols, ld, obs, n, offsets, order, rmax, sc, sink, bitmaps,
                           visible, cells, ws, as_stream(stream));
}
