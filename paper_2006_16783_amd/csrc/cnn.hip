// Learned ranking: a small CNN that predicts a post's visibility index from
// the 64 x 64 terrain patch around it, used only as an alternative FINDMAX
// key.  Forward, backward and Adam are all here; convolutions run on MFMA
// (bf16 operands, fp32 accumulation: v_mfma_f32_16x16x16_bf16 for conv1 and
// the backward GEMMs, gfx950's v_mfma_f32_16x16x32_bf16 for the forward
// conv2 and conv3).
//
// Network (patch of 64 x 64 posts around the post):
//   input  P = bf16(float(z[clamped post] - z[centre]) * 2^-8)    64 x 64
//   conv1  4x4 stride 4, 1 -> 16, ReLU  -> H1 16 x 16 x 16 (bf16)
//   conv2  3x3 stride 2, 16 -> 16, ReLU -> H2  7 x  7 x 16 (bf16)
//   conv3  3x3 stride 2, 16 -> 32, ReLU -> H3  3 x  3 x 32 (fp32)
//   global average pool, fully connected 32 -> 1, sigmoid
// Parameters are one fp32 vector (w1, b1, w2, b2, w3, b3, wfc, bfc); conv
// weights are rounded to bf16 where they enter an MFMA.
//
// MFMA 16x16x16 operand layout (per lane l of a wavefront): A supplies row
// l%16, k = 4*(l/16)..+3; B supplies column l%16, k = 4*(l/16)..+3; the
// accumulator holds column l%16, rows 4*(l/16)..+3.  The 4x4 stride-4 first
// layer is chosen so that a patch fragment is exactly 4 contiguous posts of
// one patch row (no im2col); the forward conv2/conv3 fragments (16x16x32,
// k = 8*(l/16)..+7) are 8 contiguous channels of one input position.
#include <algorithm>
#include <type_traits>

#include "common.hpp"

namespace siting {
namespace {

typedef short s4 __attribute__((ext_vector_type(4)));
typedef short s8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef uint32_t u2v __attribute__((ext_vector_type(2)));
typedef uint32_t u4v __attribute__((ext_vector_type(4)));

// parameter offsets in the flat fp32 vector
constexpr int OW1 = 0, OB1 = 256, OW2 = 272, OB2 = 2576, OW3 = 2592, OB3 = 7200, OWFC = 7232,
              OBFC = 7264, NPARAMS = 7265;
constexpr int kPatch = 64;
// wavefronts per workgroup: training stages a tile per wavefront; scoring
// shares one tile among the workgroup's wavefronts (two workgroups per CU)
constexpr int kTrainWaves = 4, kScoreWaves = 4;
template <bool kTrain>
constexpr int fwd_waves() { return kTrain ? kTrainWaves : kScoreWaves; }
// per-wavefront LDS: conv1 and conv2 activations, 16-byte entries of 8
// bf16 channels (two entries per position).  H1 rows are 20 entries (16
// columns and 4 of padding): two rows apart is then 8 entries (128 bytes)
// apart modulo 256, so the two rows that one 16-lane group of conv2 reads
// fall in different banks.
constexpr int kH1Row = 20;
constexpr int kH1Rows = 16;
constexpr int kH1Chunk = kH1Rows * kH1Row;
constexpr int kH1Bytes = 2 * kH1Chunk * 16;
// H2 keeps the 7 valid rows of conv2's 8 x 8 output grid
constexpr int kH2Chunk = 7 * 8;
constexpr int kH2Bytes = 2 * kH2Chunk * 16;
constexpr int kWaveLdsBytes = kH1Bytes + kH2Bytes;
// Terrain tile row pitch in posts: at least the width and 2 modulo 4, so
// rows start 4-byte aligned and consecutive rows are an odd number of
// dwords apart.  conv1's 32-lane half reads two consecutive rows, 16 lanes
// each two dwords apart: the odd offset puts the two rows in opposite
// banks.
__host__ __device__ constexpr int tile_pitch(int w) { return w + ((2 - w) & 3); }
constexpr int kTrainPitch = tile_pitch(kPatch);
// Scoring tiles cover BL x BL cells with BL * stride <= 64, so a tile side
// is at most 127 posts and the pitch is one constant (row offsets become
// instruction immediates).
constexpr int kScoreSpan = 64;
constexpr int kScorePitch = tile_pitch(kScoreSpan + kPatch - 1);

__device__ __forceinline__ short bf16_bits(float f)
{
    __bf16 h = (__bf16)f;  // round to nearest even
    return __builtin_bit_cast(short, h);
}
__device__ __forceinline__ float bf16_float(uint16_t b)
{
    return __uint_as_float((uint32_t)b << 16);
}
typedef float f2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
typedef short sh2 __attribute__((ext_vector_type(2)));
// two floats to two bf16 (round to nearest even) in one packed conversion
__device__ __forceinline__ uint32_t pk_bf16(float a, float b)
{
    const bf2 h = __builtin_convertvector(f2{a, b}, bf2);
    return __builtin_bit_cast(uint32_t, h);
}
__device__ __forceinline__ s4 pack4(float a, float b, float c, float d)
{
    const uint32_t lo = pk_bf16(a, b), hi = pk_bf16(c, d);
    return __builtin_bit_cast(s4, (uint64_t)lo | ((uint64_t)hi << 32));
}
// ReLU of two bf16 given as bits: a negative bf16 (sign bit set) is a
// negative int16, so a packed int16 maximum with 0 zeroes it and keeps the
// rest (ReLU then rounding equals rounding then ReLU)
__device__ __forceinline__ uint32_t relu_bf16x2(uint32_t v)
{
    const sh2 x = __builtin_bit_cast(sh2, v);
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(x, sh2{0, 0}));
}
// Orders this wavefront's LDS writes before its later LDS reads by other
// lanes of the same wavefront.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// 8 consecutive bf16 at a 16-byte aligned LDS address (one 16-byte read,
// taken as the fragment's bits unchanged)
__device__ __forceinline__ s8 lds_frag8(const unsigned char *p)
{
    return __builtin_bit_cast(s8, *reinterpret_cast<const u4v *>(p));
}
// 8 consecutive fp32 weights as a bf16 fragment
__device__ __forceinline__ s8 pack8(const float *w)
{
    return __builtin_bit_cast(s8, u4v{pk_bf16(w[0], w[1]), pk_bf16(w[2], w[3]),
                                      pk_bf16(w[4], w[5]), pk_bf16(w[6], w[7])});
}

// wavefront max of non-negative ints and sum of floats on DPP row moves
// (no LDS); the result is taken from the last lane
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v)
{
    uint32_t w;
    w = dpp_move<0x111, 0xF>(v); v = w > v ? w : v;
    w = dpp_move<0x112, 0xF>(v); v = w > v ? w : v;
    w = dpp_move<0x114, 0xF>(v); v = w > v ? w : v;
    w = dpp_move<0x118, 0xF>(v); v = w > v ? w : v;
    w = dpp_move<0x142, 0xA>(v); v = w > v ? w : v;
    w = dpp_move<0x143, 0xC>(v); v = w > v ? w : v;
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}
__device__ __forceinline__ float wave_sum_f32(float v)
{
    v += __uint_as_float(dpp_move<0x111, 0xF>(__float_as_uint(v)));
    v += __uint_as_float(dpp_move<0x112, 0xF>(__float_as_uint(v)));
    v += __uint_as_float(dpp_move<0x114, 0xF>(__float_as_uint(v)));
    v += __uint_as_float(dpp_move<0x118, 0xF>(__float_as_uint(v)));
    v += __uint_as_float(dpp_move<0x142, 0xA>(__float_as_uint(v)));
    v += __uint_as_float(dpp_move<0x143, 0xC>(__float_as_uint(v)));
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// logistic function; the hardware reciprocal (1 ulp) in place of a
// correctly rounded division (every caller uses this one definition)
__device__ __forceinline__ float sigmoid_f32(float y)
{
    return __builtin_amdgcn_rcpf(1.0f + __expf(-y));
}

__device__ __forceinline__ f4 mfma(s4 a, s4 b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
// gfx950's double-K form: per lane k = 8*(l/16)..+7 of A's row l%16 and of
// B's column l%16; the accumulator layout is the 16x16x16 one
__device__ __forceinline__ f4 mfma32(s8 a, s8 b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a),
                                                   __builtin_bit_cast(bf8, b), c, 0, 0, 0);
}

// ----------------------------------------------------------------- forward
// One wavefront per post.  kTrain: posts are given centres and every
// activation is stored for the backward pass; otherwise the terrain is cut
// into stride x stride cells, each scored at its highest post, a workgroup
// shares one staged terrain tile among BL x BL cells, and the prediction is
// written per cell.
struct FwdArgs {
    const float *params;
    const int16_t *z;
    int64_t nrows, ncols, ld;
    // train mode
    const int64_t *centres;
    int64_t nposts;
    uint16_t *Pst, *H1st, *H2st;
    float *H3st, *gst, *yst;
    // score mode: tiles of BL x BL cells, one per workgroup, row-major
    int stride, BL;
    int64_t lat_r, lat_c, blocks_c;
    // ceil(2^20 / BL) and ceil(2^20 / stride): x / BL = (x * bl_inv) >> 20
    // exactly for x < BL^2 (BL <= 64), likewise for stride
    uint32_t bl_inv, st_inv;
    float *score;
};

template <bool kTrain>
__global__ __launch_bounds__(64 * fwd_waves<kTrain>())
__attribute__((amdgpu_waves_per_eu(2, 2))) void
cnn_fwd_kernel(FwdArgs A)
{
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int kFwdWaves = fwd_waves<kTrain>();
    const int lane = threadIdx.x & 63;
    // the wavefront index as a uniform value: per-post bookkeeping (cell,
    // highest post, patch origin) then stays in scalar registers
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lo = lane & 15, hi = lane >> 4;
    // per-wavefront activations in 16-byte entries of 8 channels:
    //   H1 [chunk 2][row 16][column 16: even columns, then odd; 4 pad]
    //   H2 [chunk 2][row 7][column 8] (column 7 unused)
    // chunk c holds channels 8c..8c+7.  An x32 fragment is one entry; the
    // 3x3 stride-2 conv2 reads input columns 2tx+kx, which this column
    // order makes consecutive in tx.
    unsigned char *H1 = smem + wave * kWaveLdsBytes;
    unsigned char *H2 = H1 + kH1Bytes;
    int16_t *tile = reinterpret_cast<int16_t *>(smem + kFwdWaves * kWaveLdsBytes);

    // weights as bf16 fragments and per-lane biases.  Scoring moves the
    // input's 2^-8 scale into w1: a power-of-two factor commutes with bf16
    // rounding and with the exact products, so the accumulators are the same
    // bits (training keeps the scaled patch, which its backward pass reads).
    // conv1 and conv2 run transposed (weights as the row operand, channels x
    // positions); conv3 runs positions x channels.  An x32 fragment spans two
    // taps: lanes with hi < 2 take tap 2j, the others tap 2j+1 (tap 9 is a
    // zero weight read over tap 8's activations).
    const float *p = A.params;
    const float w1s = kTrain ? 1.0f : 0.00390625f;
    const s4 bw1 = pack4(p[OW1 + lo * 16 + hi * 4 + 0] * w1s, p[OW1 + lo * 16 + hi * 4 + 1] * w1s,
                         p[OW1 + lo * 16 + hi * 4 + 2] * w1s, p[OW1 + lo * 16 + hi * 4 + 3] * w1s);
    const int half = hi >> 1, ci0 = 8 * (hi & 1);
    s8 aw2[5], bw3[5][2];
#pragma unroll
    for (int j = 0; j < 5; j++) {
        const int tap = 2 * j + half;
        const bool real = tap < 9;
        aw2[j] = real ? pack8(p + OW2 + lo * 144 + tap * 16 + ci0) : s8{};
#pragma unroll
        for (int nt = 0; nt < 2; nt++)
            bw3[j][nt] = real ? pack8(p + OW3 + (nt * 16 + lo) * 144 + tap * 16 + ci0) : s8{};
    }
    const f4 b1v = {p[OB1 + 4 * hi], p[OB1 + 4 * hi + 1], p[OB1 + 4 * hi + 2], p[OB1 + 4 * hi + 3]};
    const f4 b2v = {p[OB2 + 4 * hi], p[OB2 + 4 * hi + 1], p[OB2 + 4 * hi + 2], p[OB2 + 4 * hi + 3]};
    const float b3[2] = {p[OB3 + lo], p[OB3 + 16 + lo]};
    const float wfc[2] = {p[OWFC + lo], p[OWFC + 16 + lo]};
    const float bfc = p[OBFC];

    // per-lane LDS byte offsets, the same for every post
    // conv1 output: channels 4hi..4hi+3 of column lo (row oy adds
    // oy * kH1Row entries)
    const uint32_t w1off = ((hi >> 1) * kH1Chunk + (lo & 1) * 8 + (lo >> 1)) * 16 + (hi & 1) * 8;
    // conv2 runs on an 8 x 8 output grid (row 7 and column 7 discarded):
    // tile t is rows 2t, 2t+1, lane lo is row 2t + lo/8, column lo%8.
    // Output row 7 reads the inputs of row 6 (it is discarded).
    uint32_t base2[4], toff2[5];
#pragma unroll
    for (int t = 0; t < 4; t++) {
        const int ty = 2 * t + (lo >> 3) > 6 ? 6 : 2 * t + (lo >> 3), tx = lo & 7;
        base2[t] = ((hi & 1) * kH1Chunk + 2 * ty * kH1Row + tx) * 16;
    }
#pragma unroll
    for (int j = 0; j < 5; j++) {
        const int tap = 2 * j + half > 8 ? 8 : 2 * j + half;
        const int ky = tap / 3, kx = tap - 3 * ky;
        toff2[j] = (ky * kH1Row + (kx == 1 ? 8 : kx == 2 ? 1 : 0)) * 16;
    }
    // conv2 output: channels 4hi..4hi+3 of grid position 16t+lo (t adds
    // 16 entries)
    const uint32_t w2off = ((hi >> 1) * kH2Chunk + lo) * 16 + (hi & 1) * 8;
    // conv3 input: position min(lo, 8) of the 3 x 3 output, tap of step j
    uint32_t off3[5];
    {
        const int m = lo > 8 ? 8 : lo;
        const int oy = m / 3, ox = m - oy * 3;
#pragma unroll
        for (int j = 0; j < 5; j++) {
            const int tap = 2 * j + half > 8 ? 8 : 2 * j + half;
            const int ky = tap / 3, kx = tap - 3 * ky;
            off3[j] = ((hi & 1) * kH2Chunk + (2 * oy + ky) * 8 + 2 * ox + kx) * 16;
        }
    }

    // the post a lane tests in the highest-post search of a cell of at most
    // 64 posts
    constexpr int tp = kTrain ? kTrainPitch : kScorePitch;  // tile row pitch in posts
    const int e1 = !kTrain && lane < A.stride * A.stride ? lane : 0;
    const int hr = kTrain ? 0 : e1 / A.stride, hc = kTrain ? 0 : e1 - hr * A.stride;
    const int hoff = hr * tp + hc;

    // tile geometry
    int tw = kPatch, th = kPatch;  // tile width/height in posts
    int64_t ty0 = 0, tx0 = 0;      // global post of tile (0,0) (unclamped)
    int nloc = 1;                  // posts handled by this workgroup
    int64_t bi = 0, bj = 0;        // this workgroup's block of cells
    bool narrow = false;           // the tile's elevation range is <= 32767
    if (!kTrain) {
        bi = blockIdx.x / A.blocks_c;
        bj = blockIdx.x - bi * A.blocks_c;
        // patches are centred on the highest post of each cell: up to
        // stride-1 posts past the cell corner
        tw = th = A.BL * A.stride + kPatch - 1;
        ty0 = bi * A.BL * A.stride - kPatch / 2;
        tx0 = bj * A.BL * A.stride - kPatch / 2;
        // stage the clamped tile once for the whole workgroup: rows by
        // wavefronts, columns by lanes, several rows' loads in flight at
        // once.  Interior tiles of an even-pitch terrain move dwords (two
        // posts); others clamp post by post.  Both track the tile's
        // elevation range.
        const int ndw = (tw + 1) >> 1;
        const bool dwords = ty0 >= 0 && tx0 >= 0 && ty0 + th <= A.nrows &&
                            tx0 + 2 * ndw <= A.ncols && ((A.ld | tx0) & 1) == 0 &&
                            (reinterpret_cast<uintptr_t>(A.z) & 3) == 0;
        sh2 zmax = {-32768, -32768}, zmin = {32767, 32767};
        if (dwords) {
            // lane = dword column; this wavefront's rows are kFwdWaves apart
            const bool lv = lane < ndw;
            const int64_t rstep = (int64_t)kFwdWaves * (A.ld >> 1);
            const uint32_t *zrow =
                reinterpret_cast<const uint32_t *>(A.z + (ty0 + wave) * A.ld + tx0) + lane;
            for (int r0 = wave; r0 < th; r0 += 8 * kFwdWaves) {
                uint32_t v[8];
#pragma unroll
                for (int u = 0; u < 8; u++) {
                    const int r = r0 + u * kFwdWaves;
                    v[u] = (r < th && lv) ? zrow[u * rstep] : 0u;
                }
#pragma unroll
                for (int u = 0; u < 8; u++) {
                    const int r = r0 + u * kFwdWaves;
                    if (r < th && lv) {
                        *reinterpret_cast<uint32_t *>(tile + r * tp + 2 * lane) = v[u];
                        const sh2 x = __builtin_bit_cast(sh2, v[u]);
                        zmax = __builtin_elementwise_max(zmax, x);
                        zmin = __builtin_elementwise_min(zmin, x);
                    }
                }
                zrow += 8 * rstep;
            }
        } else {
            for (int r0 = wave; r0 < th; r0 += 4 * kFwdWaves) {
                int16_t v[4][2];
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    const int r = r0 + u * kFwdWaves;
                    int64_t gy = ty0 + r;
                    gy = gy < 0 ? 0 : gy > A.nrows - 1 ? A.nrows - 1 : gy;
                    const int16_t *src = A.z + gy * A.ld;
#pragma unroll
                    for (int cc = 0; cc < 2; cc++) {
                        const int c = lane + 64 * cc;
                        int64_t gx = tx0 + c;
                        gx = gx < 0 ? 0 : gx > A.ncols - 1 ? A.ncols - 1 : gx;
                        v[u][cc] = (r < th && c < tw) ? src[gx] : (int16_t)0;
                    }
                }
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    const int r = r0 + u * kFwdWaves;
#pragma unroll
                    for (int cc = 0; cc < 2; cc++) {
                        const int c = lane + 64 * cc;
                        if (r < th && c < tw) {
                            tile[r * tp + c] = v[u][cc];
                            const sh2 x = {v[u][cc], v[u][cc]};
                            zmax = __builtin_elementwise_max(zmax, x);
                            zmin = __builtin_elementwise_min(zmin, x);
                        }
                    }
                }
            }
        }
        // workgroup range: per-wave maxima of z + 32768 and 32767 - z in
        // four slots past the tile
        uint32_t *slots = reinterpret_cast<uint32_t *>(tile + th * tp);
        const int lmax = zmax.x > zmax.y ? zmax.x : zmax.y, lmin = zmin.x < zmin.y ? zmin.x : zmin.y;
        const uint32_t wmax = wave_max_u32((uint32_t)(lmax + 32768));
        const uint32_t wmin = wave_max_u32((uint32_t)(32767 - lmin));
        if (lane == 0) {
            slots[2 * wave] = wmax;
            slots[2 * wave + 1] = wmin;
        }
        __syncthreads();
        uint32_t gmax = 0, gmin = 0;
#pragma unroll
        for (int k = 0; k < kFwdWaves; k++) {
            gmax = slots[2 * k] > gmax ? slots[2 * k] : gmax;
            gmin = slots[2 * k + 1] > gmin ? slots[2 * k + 1] : gmin;
        }
        // every difference to a centre fits 16 bits
        narrow = (int)gmax + (int)gmin - 65535 <= 32767;
        nloc = A.BL * A.BL;
    } else {
        tile += wave * kPatch * kTrainPitch;
    }

    const int64_t nwork = kTrain ? A.nposts : nloc;
    const int64_t step = kTrain ? (int64_t)gridDim.x * kFwdWaves : kFwdWaves;
    const int64_t first = kTrain ? (int64_t)blockIdx.x * kFwdWaves + wave : wave;
    for (int64_t w = first; w < nwork; w += step) {
        // ---- locate the post and its patch origin inside `tile`
        int64_t pid, cy, cx;
        int or_ = 0, oc = 0;  // patch origin in the tile
        if (kTrain) {
            pid = w;
            const int64_t c = A.centres[pid];
            cy = c / A.ncols;
            cx = c - cy * A.ncols;
            // stage this post's clamped 64 x 64 window
            for (int r = 0; r < kPatch; r++) {
                int64_t gy = cy - kPatch / 2 + r, gx = cx - kPatch / 2 + lane;
                gy = gy < 0 ? 0 : gy > A.nrows - 1 ? A.nrows - 1 : gy;
                gx = gx < 0 ? 0 : gx > A.ncols - 1 ? A.ncols - 1 : gx;
                tile[r * kTrainPitch + lane] = A.z[gy * A.ld + gx];
            }
            wave_lds_sync();
        } else {
            const int wi = (int)w;  // < BL * BL
            const int py = (int)(((uint32_t)wi * A.bl_inv) >> 20), px = wi - py * A.BL;
            // cell lattice indices fit 31 bits (the lattice is at most the
            // terrain, whose side is below 2^31)
            const int li = (int)bi * A.BL + py, lj = (int)bj * A.BL + px;
            if (li >= (int)A.lat_r || lj >= (int)A.lat_c)
                continue;
            pid = (int64_t)li * A.lat_c + lj;
            // highest post of the cell (elevation desc, index asc): one wave
            // max over packed (elevation, ~row-major position) keys
            const int ss = A.stride * A.stride;
            const int cell0 = (py * A.stride + kPatch / 2) * tp + px * A.stride + kPatch / 2;
            int best = -1;
            if (ss <= 64) {
                // one post per lane (row hr, column hc of the cell)
                // rows and columns of the cell inside the terrain (uniform)
                const int64_t rl64 = A.nrows - (int64_t)li * A.stride;
                const int64_t cl64 = A.ncols - (int64_t)lj * A.stride;
                const int rl = rl64 < 64 ? (int)rl64 : 64, cl = cl64 < 64 ? (int)cl64 : 64;
                const bool ok = lane < ss && hr < rl && hc < cl;
                const int v = tile[cell0 + hoff];
                best = ok ? ((v + 32768) << 12) | (4095 - e1) : -1;
            } else {
                for (int e = lane; e < ss; e += 64) {
                    const int r = e / A.stride, c = e - r * A.stride;
                    if ((int64_t)li * A.stride + r < A.nrows && (int64_t)lj * A.stride + c < A.ncols) {
                        const int v = tile[cell0 + r * tp + c];
                        const int key = ((v + 32768) << 12) | (4095 - e);
                        best = key > best ? key : best;
                    }
                }
            }
            // every key is positive (the cell has a post), so the zeros the
            // row moves shift in never win
            best = (int)wave_max_u32((uint32_t)(best < 0 ? 0 : best));
            const int e = 4095 - (best & 4095);
            const int r = (int)(((uint32_t)e * A.st_inv) >> 20), c = e - r * A.stride;
            cy = (int64_t)li * A.stride + r;
            cx = (int64_t)lj * A.stride + c;
            or_ = py * A.stride + r;
            oc = px * A.stride + c;
        }
        const int zc = tile[(or_ + kPatch / 2) * tp + oc + kPatch / 2];

        // ---- conv1: one MFMA per output row oy (16 output columns).  The
        // four posts of a fragment are two dwords: rows start dword-aligned
        // (tp is even), so they are aligned when oc is even and otherwise
        // take three dwords shifted by one post.  All rows are read before
        // the first H1 write, so that the compiler may overlap one row's
        // conversion with another's MFMA (the LDS writes would otherwise
        // order every later read).  With a narrow tile the differences are
        // formed as packed 16-bit integers (exact there) and converted from
        // 16 bits, the same values as the 32-bit path.  Row 15 feeds no
        // conv2 output: scoring skips it, training computes it for the
        // stored activations.
        const uint32_t zc2 = (uint32_t)(uint16_t)zc * 0x10001u;
        auto conv1 = [&](auto odd, auto nar) {
            constexpr bool kOdd = decltype(odd)::value;
            constexpr bool kNarrow = decltype(nar)::value;
            constexpr int NR = kTrain ? 16 : 15;
            const int16_t *src0 = tile + (or_ + hi) * tp + oc + 4 * lo;
            uint32_t P01[NR], P23[NR];
#pragma unroll
            for (int oy = 0; oy < NR; oy++) {
                const int16_t *src = src0 + 4 * oy * tp;
                if (!kOdd) {
                    const uint32_t *q = reinterpret_cast<const uint32_t *>(src);
                    P01[oy] = q[0];
                    P23[oy] = q[1];
                } else {
                    const uint32_t *q = reinterpret_cast<const uint32_t *>(src - 1);
                    const uint32_t d0 = q[0], d1 = q[1], d2 = q[2];
                    P01[oy] = __builtin_amdgcn_alignbyte(d1, d0, 2);
                    P23[oy] = __builtin_amdgcn_alignbyte(d2, d1, 2);
                }
            }
            // four rows at a time: four independent MFMAs in flight
#pragma unroll
            for (int g = 0; g < NR; g += 4) {
                f4 c[4];
#pragma unroll
                for (int u = 0; u < 4 && g + u < NR; u++) {
                    const int oy = g + u;
                    const uint32_t p01 = P01[oy], p23 = P23[oy];
                    // elevation differences in units of 256 m (exact
                    // power-of-two scale)
                    constexpr float kScale = kTrain ? 0.00390625f : 1.0f;
                    float v0, v1, v2, v3;
                    if (kNarrow) {
                        const sh2 d01 = __builtin_bit_cast(sh2, p01) - __builtin_bit_cast(sh2, zc2);
                        const sh2 d23 = __builtin_bit_cast(sh2, p23) - __builtin_bit_cast(sh2, zc2);
                        v0 = (float)d01.x * kScale;
                        v1 = (float)d01.y * kScale;
                        v2 = (float)d23.x * kScale;
                        v3 = (float)d23.y * kScale;
                    } else {
                        v0 = (float)((int)(int16_t)(p01 & 0xFFFFu) - zc) * kScale;
                        v1 = (float)((int)(int16_t)(p01 >> 16) - zc) * kScale;
                        v2 = (float)((int)(int16_t)(p23 & 0xFFFFu) - zc) * kScale;
                        v3 = (float)((int)(int16_t)(p23 >> 16) - zc) * kScale;
                    }
                    const uint64_t a = (uint64_t)pk_bf16(v0, v1) | ((uint64_t)pk_bf16(v2, v3) << 32);
                    if (kTrain)
                        *reinterpret_cast<uint64_t *>(A.Pst + pid * 4096 + (4 * oy + hi) * 64 + 4 * lo) = a;
                    // the lane gets channels 4hi..4hi+3 of position (oy, lo);
                    // the bias is the accumulator's initial value
                    c[u] = mfma(bw1, __builtin_bit_cast(s4, a), b1v);
                }
#pragma unroll
                for (int u = 0; u < 4 && g + u < NR; u++) {
                    const int oy = g + u;
                    // ReLU on the rounded bf16 pairs
                    const uint32_t h01 = relu_bf16x2(pk_bf16(c[u][0], c[u][1]));
                    const uint32_t h23 = relu_bf16x2(pk_bf16(c[u][2], c[u][3]));
                    *reinterpret_cast<u2v *>(H1 + w1off + oy * kH1Row * 16) = u2v{h01, h23};
                    if (kTrain)
                        *reinterpret_cast<u2v *>(A.H1st + (pid * 256 + oy * 16 + lo) * 16 + 4 * hi) =
                            u2v{h01, h23};
                }
            }
        };
        if (narrow) {
            if (oc & 1)
                conv1(std::true_type{}, std::true_type{});
            else
                conv1(std::false_type{}, std::true_type{});
        } else {
            if (oc & 1)
                conv1(std::true_type{}, std::false_type{});
            else
                conv1(std::false_type{}, std::false_type{});
        }
        wave_lds_sync();

        // ---- conv2 (transposed): the 7 x 7 outputs in 4 tiles of 16 grid
        // positions, 9 taps of 16 channels in 5 x32 steps; the four tiles'
        // accumulations interleaved (independent MFMA chains)
        {
            f4 c2[4] = {b2v, b2v, b2v, b2v};
#pragma unroll
            for (int j = 0; j < 5; j++) {
#pragma unroll
                for (int t = 0; t < 4; t++) {
                    const s8 b = lds_frag8(H1 + base2[t] + toff2[j]);
                    c2[t] = mfma32(aw2[j], b, c2[t]);
                }
            }
#pragma unroll
            for (int t = 0; t < 4; t++) {
                const uint32_t h01 = relu_bf16x2(pk_bf16(c2[t][0], c2[t][1]));
                const uint32_t h23 = relu_bf16x2(pk_bf16(c2[t][2], c2[t][3]));
                const int ty = 2 * t + (lo >> 3), tx = lo & 7;
                if (ty < 7)
                    *reinterpret_cast<u2v *>(H2 + w2off + t * 256) = u2v{h01, h23};
                if (kTrain && ty < 7 && tx < 7)
                    *reinterpret_cast<u2v *>(A.H2st + (pid * 49 + ty * 7 + tx) * 16 + 4 * hi) =
                        u2v{h01, h23};
            }
        }
        wave_lds_sync();
        // ---- conv3: 9 output positions, 2 column tiles of 16 channels
        f4 c3[2] = {{b3[0], b3[0], b3[0], b3[0]}, {b3[1], b3[1], b3[1], b3[1]}};
#pragma unroll
        for (int j = 0; j < 5; j++) {
            const s8 a = lds_frag8(H2 + off3[j]);
            c3[0] = mfma32(a, bw3[j][0], c3[0]);
            c3[1] = mfma32(a, bw3[j][1], c3[1]);
        }
        // ---- ReLU, global average pool over the 9 positions, FC: each
        // lane's share of the FC sum over its channels and positions, then
        // one wavefront sum (the same order in both modes); training also
        // keeps the pooled features
        float part = 0.f;
#pragma unroll
        for (int nt = 0; nt < 2; nt++) {
            float s = 0.f;
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const int pos = 4 * hi + i;
                // ReLU as an integer maximum of the bits (negative floats
                // are negative integers)
                const float h = __int_as_float(max(__float_as_int(c3[nt][i]), 0));
                if (pos < 9) {
                    s += h;
                    if (kTrain)
                        A.H3st[(pid * 9 + pos) * 32 + nt * 16 + lo] = h;
                }
            }
            part += wfc[nt] * s;
            if (kTrain) {
                float gs = s + __shfl_xor(s, 16, 64);
                gs += __shfl_xor(gs, 32, 64);
                if (hi == 0)
                    A.gst[pid * 32 + nt * 16 + lo] = gs * (1.0f / 9.0f);
            }
        }
        // the pool's 1/9 applied once to the sum
        const float y = wave_sum_f32(part) * (1.0f / 9.0f) + bfc;
        if (lane == 0) {
            if (kTrain)
                A.yst[pid] = y;
            else
                A.score[pid] = sigmoid_f32(y);
        }
        wave_lds_sync();
    }
}

// --------------------------------------------------------------- backward
// Head: p = sigmoid(y); dL/dy of the mean squared error; the gradient of
// the pooled features spread over the 9 conv3 positions through the ReLU.
__global__ void cnn_head_bwd(const float *__restrict__ params, const float *__restrict__ y,
                             const float *__restrict__ labels, const float *__restrict__ H3,
                             int64_t B, float *__restrict__ dy, float *__restrict__ sq,
                             uint16_t *__restrict__ dA3)
{
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B)
        return;
    const float pr = sigmoid_f32(y[b]);
    const float e = pr - labels[b];
    const float d = 2.0f * e / (float)B * pr * (1.0f - pr);
    dy[b] = d;
    sq[b] = e * e;
    for (int pos = 0; pos < 9; pos++)
        for (int co = 0; co < 32; co++) {
            const float h = H3[(b * 9 + pos) * 32 + co];
            const float v = h > 0.f ? d * params[OWFC + co] / 9.0f : 0.f;
            dA3[(b * 9 + pos) * 32 + co] = (uint16_t)bf16_bits(v);
        }
}

// Generic MFMA "gather GEMM": C[m][n] = sum_k A(m, k) * B(k, n) over k-blocks
// of 16, one wavefront per (16 x 16 tile, k-split); partial results go to
// out[split][m][n] and are summed later in a fixed order (deterministic).
template <class Op>
__global__ __launch_bounds__(256) void gemm_kernel(Op op)
{
    const int lane = threadIdx.x & 63, lo = lane & 15, hi = lane >> 4;
    const int64_t wg = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int64_t ntile = (int64_t)op.MT * op.NT;
    if (wg >= ntile * op.S)
        return;
    const int tile = (int)(wg % ntile), split = (int)(wg / ntile);
    const int mt = tile / op.NT, nt = tile % op.NT;
    const int64_t kb0 = (int64_t)split * op.KS;
    const int64_t kb1 = kb0 + op.KS < op.KB ? kb0 + op.KS : op.KB;
    f4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int64_t kb = kb0; kb < kb1; kb++) {
        const int64_t k = kb * 16 + 4 * hi;
        acc = mfma(op.a(mt * 16 + lo, k), op.b(k, nt * 16 + lo), acc);
    }
#pragma unroll
    for (int i = 0; i < 4; i++)
        op.store(split, mt * 16 + 4 * hi + i, nt * 16 + lo, acc[i]);
}

__device__ __forceinline__ s4 load4_strided(const uint16_t *p, int64_t stride, int64_t valid)
{
    s4 r;
    r.x = valid > 0 ? (short)p[0] : (short)0;
    r.y = valid > 1 ? (short)p[stride] : (short)0;
    r.z = valid > 2 ? (short)p[2 * stride] : (short)0;
    r.w = valid > 3 ? (short)p[3 * stride] : (short)0;
    return r;
}

// backward-weight: dW[co][tap*CI + ci] = sum_rows dA[row][co] * X(row, tap, ci)
// rows = samples x output positions (OH x OH).  X gathers the layer input
// (the bf16 patch for conv1).  KW is the kernel width.
template <int OH, int CO, int IH, int CI, int KW, int STRIDE, bool kPatchIn>
struct WgradOp {
    const uint16_t *dA;  // [rows][CO] bf16
    const uint16_t *X;   // layer input, bf16: [B][IH*IH][CI] (or the patch [B][64][64])
    float *part;         // [S][CO][N]
    int64_t rows;
    int MT, NT, S;
    int64_t KB, KS;      // k-blocks in total and per split
    static constexpr int N = KW * KW * CI;
    __device__ s4 a(int m, int64_t k) const
    {
        return load4_strided(dA + k * CO + m, CO, rows - k);
    }
    __device__ s4 b(int64_t k, int n) const
    {
        const int tap = n / CI, ci = n - tap * CI;
        const int ky = tap / KW, kx = tap - ky * KW;
        short e[4];
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const int64_t row = k + i;
            if (row >= rows) {
                e[i] = 0;
                continue;
            }
            const int64_t smp = row / (OH * OH);
            const int pos = (int)(row - smp * (OH * OH));
            const int oy = pos / OH, ox = pos - oy * OH;
            const int iy = STRIDE * oy + ky, ix = STRIDE * ox + kx;
            e[i] = kPatchIn ? (short)X[smp * 4096 + iy * 64 + ix]
                            : (short)X[(smp * (IH * IH) + iy * IH + ix) * CI + ci];
        }
        return s4{e[0], e[1], e[2], e[3]};
    }
    __device__ void store(int split, int m, int n, float v) const
    {
        if (m < CO && n < N)
            part[((int64_t)split * CO + m) * N + n] = v;
    }
};

// backward-data columns: col[row][tap*CI + ci] = sum_co dA[row][co] * W[co][tap][ci]
template <int CO, int CI, int KW>
struct ColOp {
    const uint16_t *dA;   // [rows][CO]
    const uint16_t *W;    // bf16 [CO][KW*KW][CI]
    float *col;           // [rows][N]
    int64_t rows;
    int MT, NT, S;
    int64_t KB, KS;
    static constexpr int N = KW * KW * CI;
    __device__ s4 a(int64_t m, int64_t k) const
    {
        if (m >= rows)
            return s4{0, 0, 0, 0};
        const uint16_t *p = dA + m * CO + k;
        return s4{(short)p[0], (short)p[1], (short)p[2], (short)p[3]};
    }
    __device__ s4 b(int64_t k, int n) const
    {
        return load4_strided(W + k * N + n, N, CO - k);
    }
    __device__ void store(int, int64_t m, int n, float v) const
    {
        if (m < rows)
            col[m * N + n] = v;
    }
};

// col2im gather for a 3x3 stride-2 layer: dX[s][iy][ix][ci] = sum over the
// (output position, tap) pairs reading (iy, ix), then the ReLU mask of the
// layer input, rounded to bf16 as the next MFMA consumes it.
template <int OH, int IH, int CI>
__global__ void col2im_relu(const float *__restrict__ col, const uint16_t *__restrict__ Xin,
                            int64_t B, uint16_t *__restrict__ dAin)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= B * IH * IH * CI)
        return;
    const int ci = (int)(e % CI);
    const int64_t sp = e / CI;
    const int pos = (int)(sp % (IH * IH));
    const int64_t s = sp / (IH * IH);
    const int iy = pos / IH, ix = pos - iy * IH;
    float acc = 0.f;
    for (int ky = 0; ky < 3; ky++) {
        const int ty = iy - ky;
        if (ty < 0 || (ty & 1) || (ty >> 1) >= OH)
            continue;
        for (int kx = 0; kx < 3; kx++) {
            const int tx = ix - kx;
            if (tx < 0 || (tx & 1) || (tx >> 1) >= OH)
                continue;
            const int64_t row = s * (OH * OH) + (ty >> 1) * OH + (tx >> 1);
            acc += col[row * (9 * CI) + (ky * 3 + kx) * CI + ci];
        }
    }
    const float x = bf16_float(Xin[e]);
    dAin[e] = (uint16_t)bf16_bits(x > 0.f ? acc : 0.f);
}

// Fixed-order sums: out[j] = sum_s part[s][j] (weights), and bias / head
// gradients as column sums over rows.
__global__ void sum_partials(const float *__restrict__ part, int S, int64_t n,
                             float *__restrict__ out)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n)
        return;
    float s = 0.f;
    for (int k = 0; k < S; k++)
        s += part[(int64_t)k * n + j];
    out[j] = s;
}

// column sums of a bf16 [rows][C] matrix into out[C] (one workgroup per
// column, fixed-order tree inside the workgroup)
__global__ void colsum_bf16(const uint16_t *__restrict__ m, int64_t rows, int C,
                            float *__restrict__ out)
{
    __shared__ float red[256];
    const int c = blockIdx.x;
    float s = 0.f;
    for (int64_t r = threadIdx.x; r < rows; r += 256)
        s += bf16_float(m[r * C + c]);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        out[c] = red[0];
}

// FC head gradients and the loss: dWfc[co] = sum_b dy_b g_b[co],
// dbfc = sum_b dy_b, loss = mean_b sq_b (one workgroup, fixed order).
__global__ void head_grads(const float *__restrict__ dy, const float *__restrict__ g,
                           const float *__restrict__ sq, int64_t B, float *__restrict__ grad,
                           float *__restrict__ loss)
{
    __shared__ float red[256];
    for (int j = 0; j < 34; j++) {
        float s = 0.f;
        for (int64_t b = threadIdx.x; b < B; b += 256)
            s += j < 32 ? dy[b] * g[b * 32 + j] : (j == 32 ? dy[b] : sq[b]);
        red[threadIdx.x] = s;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (threadIdx.x < w)
                red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            if (j < 32)
                grad[OWFC + j] = red[0];
            else if (j == 32)
                grad[OBFC] = red[0];
            else if (loss)
                *loss = red[0] / (float)B;
        }
        __syncthreads();
    }
}

__global__ void sigmoid_kernel(const float *__restrict__ y, int64_t n, float *__restrict__ p)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        p[i] = sigmoid_f32(y[i]);
}

__global__ void to_bf16(const float *__restrict__ x, int64_t n, uint16_t *__restrict__ y)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        y[i] = (uint16_t)bf16_bits(x[i]);
}

// Adam (Kingma & Ba) with bias correction; step counts from 1.
__global__ void adam_kernel(float *__restrict__ p, float *__restrict__ m, float *__restrict__ v,
                            const float *__restrict__ g, int64_t n, float lr, float b1, float b2,
                            float eps, float c1, float c2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ----------------------------------------------------------- workspace
struct Ws {
    uint16_t *P, *H1, *H2, *dA3, *dA2, *dA1, *wbf;
    float *H3, *g, *y, *dy, *sq, *col, *part;
    size_t bytes;
};

constexpr int kMaxSplits = 64;
constexpr int64_t kPartFloats = (int64_t)kMaxSplits * 32 * 144;

static size_t al(size_t v) { return (v + 255) & ~(size_t)255; }

static Ws ws_layout(int64_t B, void *base)
{
    Ws w{};
    size_t o = 0;
    char *c = reinterpret_cast<char *>(base);
    auto take = [&](size_t bytes) { char *p = c ? c + o : nullptr; o += al(bytes); return p; };
    w.P = (uint16_t *)take((size_t)B * 4096 * 2);
    w.H1 = (uint16_t *)take((size_t)B * 256 * 16 * 2);
    w.H2 = (uint16_t *)take((size_t)B * 49 * 16 * 2);
    w.H3 = (float *)take((size_t)B * 9 * 32 * 4);
    w.g = (float *)take((size_t)B * 32 * 4);
    w.y = (float *)take((size_t)B * 4);
    w.dy = (float *)take((size_t)B * 4);
    w.sq = (float *)take((size_t)B * 4);
    w.dA3 = (uint16_t *)take((size_t)B * 9 * 32 * 2);
    w.dA2 = (uint16_t *)take((size_t)B * 49 * 16 * 2);
    w.dA1 = (uint16_t *)take((size_t)B * 256 * 16 * 2);
    w.col = (float *)take((size_t)B * 49 * 144 * 4);
    w.part = (float *)take((size_t)kPartFloats * 4);
    w.wbf = (uint16_t *)take((size_t)NPARAMS * 2);
    w.bytes = o;
    return w;
}

template <class Op>
static int launch_gemm(Op op, hipStream_t s, const char *what)
{
    const int64_t waves = (int64_t)op.MT * op.NT * op.S;
    hipLaunchKernelGGL(gemm_kernel<Op>, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s, op);
    return check_launch(what);
}

// split count so that each wavefront does ~64 k-blocks, at most kMaxSplits
static void pick_splits(int64_t KB, int &S, int64_t &KS)
{
    S = (int)std::min<int64_t>(kMaxSplits, std::max<int64_t>(1, (KB + 63) / 64));
    KS = (KB + S - 1) / S;
}

}  // namespace
}  // namespace siting

using namespace siting;

extern "C" int siting_cnn_param_count(void) { return NPARAMS; }

extern "C" size_t siting_cnn_workspace_size(int64_t batch)
{
    if (batch < 1)
        return 0;
    return ws_layout(batch, nullptr).bytes;
}

static int check_terrain(const int16_t *z, int64_t nrows, int64_t ncols, int64_t ld,
                         const char *fn)
{
    SITING_REQUIRE(z != nullptr, "%s: NULL terrain", fn);
    SITING_REQUIRE(nrows >= 1 && ncols >= 1 && ld >= ncols, "%s: bad terrain shape", fn);
    return SITING_OK;
}

extern "C" int siting_cnn_forward(const float *params, const int16_t *z, int64_t nrows,
                                  int64_t ncols, int64_t ld, const int64_t *centres, int64_t B,
                                  float *pred, void *ws, size_t ws_bytes, void *stream)
{
    clear_error();
    const char *fn = "siting_cnn_forward";
    int rc = check_terrain(z, nrows, ncols, ld, fn);
    if (rc != SITING_OK)
        return rc;
    SITING_REQUIRE(params && centres && B >= 1, "%s: NULL pointer or empty batch", fn);
    if (!ws || ws_bytes < siting_cnn_workspace_size(B)) {
        set_error("%s: workspace of %zu bytes needed", fn, siting_cnn_workspace_size(B));
        return SITING_E_WORKSPACE;
    }
    Ws w = ws_layout(B, ws);
    FwdArgs a{};
    a.params = params; a.z = z; a.nrows = nrows; a.ncols = ncols; a.ld = ld;
    a.centres = centres; a.nposts = B;
    a.Pst = w.P; a.H1st = w.H1; a.H2st = w.H2; a.H3st = w.H3; a.gst = w.g; a.yst = w.y;
    hipStream_t s = as_stream(stream);
    const size_t lds = kTrainWaves * (kWaveLdsBytes + kPatch * kTrainPitch * 2);
    const int64_t grid = std::min<int64_t>((B + kTrainWaves - 1) / kTrainWaves,
                                           (int64_t)device_cus() * 8);
    hipLaunchKernelGGL(cnn_fwd_kernel<true>, dim3((unsigned)grid), dim3(64 * kTrainWaves), lds, s, a);
    rc = check_launch("cnn_fwd_kernel");
    if (rc != SITING_OK || !pred)
        return rc;
    hipLaunchKernelGGL(sigmoid_kernel, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, s, w.y, B,
                       pred);
    return check_launch("cnn_sigmoid");
}

extern "C" int siting_cnn_backward(const float *params, const float *labels, int64_t B,
                                   float *grad, float *loss, void *ws, size_t ws_bytes,
                                   void *stream)
{
    clear_error();
    const char *fn = "siting_cnn_backward";
    SITING_REQUIRE(params && labels && grad && B >= 1, "%s: NULL pointer or empty batch", fn);
    if (!ws || ws_bytes < siting_cnn_workspace_size(B)) {
        set_error("%s: workspace of %zu bytes needed", fn, siting_cnn_workspace_size(B));
        return SITING_E_WORKSPACE;
    }
    Ws w = ws_layout(B, ws);
    hipStream_t s = as_stream(stream);
    int rc;
    hipLaunchKernelGGL(to_bf16, dim3((NPARAMS + 255) / 256), dim3(256), 0, s, params,
                       (int64_t)NPARAMS, w.wbf);
    if ((rc = check_launch("to_bf16")) != SITING_OK)
        return rc;
    hipLaunchKernelGGL(cnn_head_bwd, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, s, params,
                       w.y, labels, w.H3, B, w.dy, w.sq, w.dA3);
    if ((rc = check_launch("cnn_head_bwd")) != SITING_OK)
        return rc;
    hipLaunchKernelGGL(head_grads, dim3(1), dim3(256), 0, s, w.dy, w.g, w.sq, B, grad, loss);
    if ((rc = check_launch("head_grads")) != SITING_OK)
        return rc;

    // ---- conv3: weights, bias, then data gradient into H2's positions
    {
        WgradOp<3, 32, 7, 16, 3, 2, false> op{};
        op.dA = w.dA3; op.X = w.H2; op.part = w.part; op.rows = B * 9;
        op.MT = 2; op.NT = 9; op.KB = (op.rows + 15) / 16;
        pick_splits(op.KB, op.S, op.KS);
        if ((rc = launch_gemm(op, s, "wgrad3")) != SITING_OK)
            return rc;
        hipLaunchKernelGGL(sum_partials, dim3((32 * 144 + 255) / 256), dim3(256), 0, s, w.part,
                           op.S, (int64_t)32 * 144, grad + OW3);
        if ((rc = check_launch("sum_partials")) != SITING_OK)
            return rc;
        hipLaunchKernelGGL(colsum_bf16, dim3(32), dim3(256), 0, s, w.dA3, B * 9, 32, grad + OB3);
        if ((rc = check_launch("colsum_bf16")) != SITING_OK)
            return rc;
        ColOp<32, 16, 3> cop{};
        cop.dA = w.dA3; cop.W = w.wbf + OW3; cop.col = w.col; cop.rows = B * 9;
        cop.MT = (int)((cop.rows + 15) / 16); cop.NT = 9; cop.S = 1; cop.KB = 2; cop.KS = 2;
        if ((rc = launch_gemm(cop, s, "col3")) != SITING_OK)
            return rc;
        const int64_t n2 = B * 49 * 16;
        hipLaunchKernelGGL((col2im_relu<3, 7, 16>), dim3((unsigned)((n2 + 255) / 256)), dim3(256),
                           0, s, w.col, w.H2, B, w.dA2);
        if ((rc = check_launch("col2im3")) != SITING_OK)
            return rc;
    }
    // ---- conv2
    {
        WgradOp<7, 16, 16, 16, 3, 2, false> op{};
        op.dA = w.dA2; op.X = w.H1; op.part = w.part; op.rows = B * 49;
        op.MT = 1; op.NT = 9; op.KB = (op.rows + 15) / 16;
        pick_splits(op.KB, op.S, op.KS);
        if ((rc = launch_gemm(op, s, "wgrad2")) != SITING_OK)
            return rc;
        hipLaunchKernelGGL(sum_partials, dim3((16 * 144 + 255) / 256), dim3(256), 0, s, w.part,
                           op.S, (int64_t)16 * 144, grad + OW2);
        if ((rc = check_launch("sum_partials")) != SITING_OK)
            return rc;
        hipLaunchKernelGGL(colsum_bf16, dim3(16), dim3(256), 0, s, w.dA2, B * 49, 16, grad + OB2);
        if ((rc = check_launch("colsum_bf16")) != SITING_OK)
            return rc;
        ColOp<16, 16, 3> cop{};
        cop.dA = w.dA2; cop.W = w.wbf + OW2; cop.col = w.col; cop.rows = B * 49;
        cop.MT = (int)((cop.rows + 15) / 16); cop.NT = 9; cop.S = 1; cop.KB = 1; cop.KS = 1;
        if ((rc = launch_gemm(cop, s, "col2")) != SITING_OK)
            return rc;
        const int64_t n1 = B * 256 * 16;
        hipLaunchKernelGGL((col2im_relu<7, 16, 16>), dim3((unsigned)((n1 + 255) / 256)),
                           dim3(256), 0, s, w.col, w.H1, B, w.dA1);
        if ((rc = check_launch("col2im2")) != SITING_OK)
            return rc;
    }
    // ---- conv1 (weights and bias only; the input needs no gradient)
    {
        WgradOp<16, 16, 64, 1, 4, 4, true> op{};
        op.dA = w.dA1; op.X = w.P; op.part = w.part; op.rows = B * 256;
        op.MT = 1; op.NT = 1; op.KB = (op.rows + 15) / 16;
        pick_splits(op.KB, op.S, op.KS);
        if ((rc = launch_gemm(op, s, "wgrad1")) != SITING_OK)
            return rc;
        hipLaunchKernelGGL(sum_partials, dim3(1), dim3(256), 0, s, w.part, op.S, (int64_t)256,
                           grad + OW1);
        if ((rc = check_launch("sum_partials")) != SITING_OK)
            return rc;
        hipLaunchKernelGGL(colsum_bf16, dim3(16), dim3(256), 0, s, w.dA1, B * 256, 16, grad + OB1);
        if ((rc = check_launch("colsum_bf16")) != SITING_OK)
            return rc;
    }
    return SITING_OK;
}

extern "C" int siting_cnn_adam(float *params, float *m, float *v, const float *grad, int64_t n,
                               int32_t step, float lr, float beta1, float beta2, float eps,
                               void *stream)
{
    clear_error();
    SITING_REQUIRE(params && m && v && grad, "siting_cnn_adam: NULL pointer");
    SITING_REQUIRE(n >= 1 && step >= 1, "siting_cnn_adam: n and step must be >= 1");
    SITING_REQUIRE(lr > 0.f && beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f &&
                       eps > 0.f, "siting_cnn_adam: bad hyper-parameters");
    const float c1 = 1.f - powf(beta1, (float)step), c2 = 1.f - powf(beta2, (float)step);
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                       as_stream(stream), params, m, v, grad, n, lr, beta1, beta2, eps, c1, c2);
    return check_launch("adam_kernel");
}

extern "C" int siting_cnn_score_terrain(const float *params, const int16_t *z, int64_t nrows,
                                        int64_t ncols, int64_t ld, int32_t stride, float *score,
                                        void *stream)
{
    clear_error();
    const char *fn = "siting_cnn_score_terrain";
    int rc = check_terrain(z, nrows, ncols, ld, fn);
    if (rc != SITING_OK)
        return rc;
    SITING_REQUIRE(params && score, "%s: NULL pointer", fn);
    SITING_REQUIRE(stride >= 1 && stride <= 64, "%s: stride %d outside 1..64", fn, stride);
    FwdArgs a{};
    a.params = params; a.z = z; a.nrows = nrows; a.ncols = ncols; a.ld = ld;
    a.stride = stride;
    // cells per tile side: BL * stride <= 64 posts plus the 63-post patch
    // margin (two workgroups per CU at every stride)
    a.BL = std::max(1, kScoreSpan / stride);
    a.bl_inv = ((1u << 20) + (uint32_t)a.BL - 1) / (uint32_t)a.BL;
    a.st_inv = ((1u << 20) + (uint32_t)stride - 1) / (uint32_t)stride;
    a.lat_r = (nrows + stride - 1) / stride;
    a.lat_c = (ncols + stride - 1) / stride;
    const int64_t blocks_r = (a.lat_r + a.BL - 1) / a.BL;
    a.blocks_c = (a.lat_c + a.BL - 1) / a.BL;
    a.score = score;
    const int tw = a.BL * stride + kPatch - 1;
    const size_t lds = kScoreWaves * kWaveLdsBytes + (size_t)tw * kScorePitch * 2 + 8 * kScoreWaves;
    if ((int64_t)lds > kernel_max_dynamic_lds(reinterpret_cast<const void *>(&cnn_fwd_kernel<false>))) {
        set_error("%s: tile does not fit in LDS", fn);
        return SITING_E_UNSUPPORTED;
    }
    const int64_t grid = blocks_r * a.blocks_c;
    if (grid > INT32_MAX) {
        set_error("%s: terrain too large", fn);
        return SITING_E_UNSUPPORTED;
    }
    hipLaunchKernelGGL(cnn_fwd_kernel<false>, dim3((unsigned)grid), dim3(64 * kScoreWaves), lds,
                       as_stream(stream), a);
    return check_launch("cnn_fwd_kernel");
}
