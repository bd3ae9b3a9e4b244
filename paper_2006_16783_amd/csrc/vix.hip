// VIX: estimated visibility index of every post from K random receivers in
// its ROI disk (stage Vix of the siting process).
//
// Layout: the terrain is cut into T x T post tiles; a workgroup stages its
// tile plus a halo of H = R + s - 1 posts ((T+2H)^2 int16; s LOS steps per
// block) in LDS when that fits, so every line-of-sight sample is an LDS read
// and a block's steps past the end of its line (discarded) need no mask;
// otherwise (large ROI) it reads the terrain through L2, masked, and tiles
// only give spatial locality.  Tiles are handed
// to XCDs in contiguous bands so that neighbouring halos share an L2.
//
// Scheduling: a line of sight ends at its first blocking sample, so test
// lengths vary from 1 to R steps (7 on average on rough terrain, while the
// visible ones run to the end).  One test per lane would leave a wavefront
// waiting for its longest test.  Instead each wavefront takes batches of 64
// posts of its tile; it draws up to 10 receivers per post into registers of
// the post's lane (the queue: row j holds draw j of every post), then its
// lanes pull tests from the queue in order, reading the entry and the post's
// offset and eye elevation from the owning lane (ds_bpermute), and a lane
// whose test ends takes the next one (ballot + prefix count).  When the queue
// runs dry the wavefront draws its next chunk or claims its next batch at
// once, while the long tests of the previous batch keep running; visible
// results go to per-post LDS counters, double-buffered by batch, so a batch's
// counts are written out once its last test has ended.  A wavefront drains
// only at the end of its tile.  Each queue iteration advances a test by a
// block of steps whose reads are all issued before any comparison, one LDS
// round trip per block.
//
// Draws: post t owns one Philox4x32-10 stream (word a = word a%4 of the
// block {t lo, a/4, t hi, 0} under key {seed lo, seed hi}); each word
// proposes one receiver, its 16-bit halves scaled to the clipped box by
// Lemire's multiply-shift with rejection (exactly uniform; full-rate 24-bit
// multiplies).  The block index sits in a counter word that the first round
// does not multiply, so that round's products depend only on the post and
// are computed once per batch.  The generator runs only when some lane of
// the wavefront has used up its block, with all lanes computing it together.
//
// Exactness: everything is integer.  At major step k of a LOS of length n
// (k*|minor| = q*n + r) the terrain sample is S = z0*n + (z1-z0)*r, computed
// as z1*n + (z1-z0)*e with e = r - n in [-n, -1] (e + |minor| >= 0 is then the
// carry of one add), and the segment is E*n + (Z-E)*k; with |z| < 2^15,
// n <= 4094 and heights <= 2^15 every term fits in int32 and the 24-bit
// multipliers are exact.
#include "common.hpp"

namespace siting {
namespace {

constexpr int kVixWaves = 16;
constexpr int kVixThreads = 64 * kVixWaves;
constexpr int kVixChunk = 10;          // draws per post per queue round
constexpr int kVixMaxAttempts = 64;    // consecutive rejections before a draw fails
constexpr int kVixMaxRoi = 4094;       // LOS lengths keep every product in int32
// queue words that hold no test: a slot not yet drawn, and a failed draw (or
// a slot past the chunk).  Their dx (32767) is no receiver's, and as signed
// words every test entry is below both.
constexpr uint32_t kEmpty = 0x7FFF7FFFu;
constexpr uint32_t kNoTest = 0x7FFF7FFEu;
// LOS steps per queue iteration: longer blocks waste the steps after a
// test's end (most tests end within a few steps), shorter ones take tests
// more often; 5 measured fastest (and its narrower halo fits a 72-post tile
// at ROI 100)
constexpr int kSPI = 5;

// Count buffers per wavefront (batches in flight) and the LDS bytes besides
// the tile: per wavefront kVixBufs x 64 8-bit visible counters (K <= 255).
constexpr int kVixBufs = 4;
constexpr int kVixWaveLds = kVixBufs * 64;

// a ^ b ^ k as one three-input bit operation (truth table 0x96); the
// compiler emits two v_xor_b32 for the plain expression
__device__ __forceinline__ uint32_t xor3_key(uint32_t a, uint32_t b, uint32_t k)
{
    return __builtin_amdgcn_bitop3_b32(a, b, k, 0x96);
}

// Philox4x32-10 block function (Salmon et al., SC'11): per round two 32x32
// products (one v_mad_u64_u32 each), their high halves mixed with the other
// counter words and the key, and the key bumped by the Weyl constants.  The
// key is wave-uniform (the seed).
__device__ __forceinline__ void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                              uint32_t k0, uint32_t k1, uint32_t out[4])
{
    constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
    for (int round = 0; round < 10; round++) {
        const uint64_t p0 = (uint64_t)M0 * c0, p1 = (uint64_t)M1 * c2;
        const uint32_t n0 = xor3_key((uint32_t)(p1 >> 32), c1, k0);
        const uint32_t n2 = xor3_key((uint32_t)(p0 >> 32), c3, k1);
        c0 = n0; c1 = (uint32_t)p1; c2 = n2; c3 = (uint32_t)p0;
        k0 += W0; k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

// 24-bit signed multiply (full rate).  Operands here are a post elevation
// (16 bits), a LOS length, step remainder or a tile pitch (< 2^13), so the
// product is exact; written out because the compiler loses those ranges.
__device__ __forceinline__ int mul_i24(int a, int b)
{
    int r;
    asm("v_mul_i32_i24 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

__device__ __forceinline__ int mad_i24(int a, int b, int c)
{
    int r;
    asm("v_mad_i32_i24 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

// the same with a wave-uniform second factor, read from a scalar register
__device__ __forceinline__ int mul_i24_s(int a, int b)
{
    int r;
    asm("v_mul_i32_i24 %0, %1, %2" : "=v"(r) : "v"(a), "s"(b));
    return r;
}

__device__ __forceinline__ int mad_i24_s(int a, int b, int c)
{
    int r;
    asm("v_mad_i32_i24 %0, %1, %2, %3" : "=v"(r) : "v"(a), "s"(b), "v"(c));
    return r;
}

// -1, 0 or 1 by the sign of a (one v_med3_i32; the compiler's form of the
// clamp is two compares and two selects)
__device__ __forceinline__ int sign3(int a)
{
    int r;
    asm("v_med3_i32 %0, %1, -1, 1" : "=v"(r) : "v"(a));
    return r;
}

// queue entry: dx and dy as the high and low 16-bit halves (two's
// complement), one byte permute
__device__ __forceinline__ uint32_t pack_test(int dx, int dy)
{
    return __builtin_amdgcn_perm((uint32_t)dx, (uint32_t)dy, 0x05040100u);
}

// LDS read at a byte address (the address includes the tile's base, so the
// load needs no add).
typedef const int16_t __attribute__((address_space(3))) lds_i16;
__device__ __forceinline__ int lds_read_i16(int addr)
{
    return *reinterpret_cast<lds_i16 *>((uintptr_t)(uint32_t)addr);
}

__device__ __forceinline__ uint32_t lane_read(int src, uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_ds_bpermute(src << 2, (int)v);
}

// kLds: terrain tile staged in LDS (else global reads).  kCount: also count
// executed LOS steps and tests, and record the lowest and highest terrain
// element offsets the kernel reads from global memory.
template <bool kLds, bool kCount>
__global__ __launch_bounds__(kVixThreads) void vix_kernel(
    const int16_t *__restrict__ z, int64_t nrows, int64_t ncols, int64_t ld, int R, int h_t,
    int h_r, int K, uint64_t seed, uint8_t *__restrict__ count, int T, int64_t tiles_r,
    int64_t tiles_c, int64_t per_xcd, int tile_bytes, int dma,
    unsigned long long *__restrict__ stats)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_batch;
    uint64_t steps = 0, tests = 0;
    // counting variant: element offsets (from z) of every global terrain read
    int64_t rd_lo = INT64_MAX, rd_hi = INT64_MIN;
    auto note = [&](int64_t o) {
        if (kCount) {
            rd_lo = o < rd_lo ? o : rd_lo;
            rd_hi = o > rd_hi ? o : rd_hi;
        }
    };
    // XCD-aware tile order: workgroup b runs on XCD b % 8; give each XCD a
    // contiguous band of tiles.
    const int64_t b = blockIdx.x;
    const int64_t t_id = (b & 7) * per_xcd + (b >> 3);
    if (t_id >= tiles_r * tiles_c)
        return;
    const int64_t r0 = (t_id / tiles_c) * T, c0 = (t_id % tiles_c) * T;
    // LDS halo: the ROI plus the steps a block can run past the end of a
    // line of sight (those reads are discarded, but stay inside the tile)
    const int H = kLds ? R + kSPI - 1 : R;
    // LDS rows hold T+2H posts starting at an even terrain column (so that
    // post pairs are dwords on both sides), padded to an even pitch
    const int pitch = T + 2 * H + 2;
    const int64_t ox = c0 - H, oxl = ox - (ox & 1), oy = r0 - H;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int16_t *tile = reinterpret_cast<int16_t *>(smem);
    // visible counts of this wavefront's batches in flight: kVixBufs buffers
    // of 64 8-bit counters, four per 32-bit word
    uint32_t *cnt = reinterpret_cast<uint32_t *>(smem + tile_bytes) + wave * (kVixBufs * 16);
    if (tid == 0)
        s_batch = 0;
    if (lane < kVixBufs * 16)
        cnt[lane] = 0;
    if (kLds) {
        const int rows = T + 2 * H;
        const int64_t gy0 = oy < 0 ? 0 : oy, gy1 = oy + rows > nrows ? nrows : oy + rows;
        if (dma) {
            // each wavefront streams its rows straight into LDS (global_load_lds:
            // lane i of a load writes the dword at the wavefront's LDS base + 4i),
            // every load of the tile in flight before the one wait below
            const bool interior = oy >= 0 && oy + rows <= nrows && oxl >= 0 && oxl + pitch <= ncols;
            const int dw_row = pitch >> 1;
            uint32_t *tdw = reinterpret_cast<uint32_t *>(tile);
            for (int lr = wave; lr < rows; lr += kVixWaves) {
                const int64_t gy = oy + lr;
                if (gy < gy0 || gy >= gy1)
                    continue;
                const int16_t *srow = z + gy * ld;
                for (int k0 = 0; k0 < dw_row; k0 += 64) {
                    const int k = k0 + lane;
                    const int64_t c = oxl + 2 * k;
                    if (k < dw_row && (interior || (c >= 0 && c < ncols))) {
                        __builtin_amdgcn_global_load_lds(
                            reinterpret_cast<const uint32_t *>(srow + c), tdw + lr * dw_row + k0, 4,
                            0, 0);
                        note(gy * ld + c);
                        note(gy * ld + c + 1);
                    }
                }
            }
            __builtin_amdgcn_s_waitcnt(0);
        } else {
            const int64_t gx0 = ox < 0 ? 0 : ox, gx1 = c0 + T + H > ncols ? ncols : c0 + T + H;
            const int w = (int)(gx1 - gx0), h = (int)(gy1 - gy0);
            for (int row = wave; row < h; row += kVixWaves) {
                const int16_t *src = z + (gy0 + row) * ld + gx0;
                int16_t *dst = tile + (gy0 + row - oy) * pitch + (gx0 - oxl);
                for (int col = lane; col < w; col += 64) {
                    dst[col] = src[col];
                    note((gy0 + row) * ld + gx0 + col);
                }
            }
        }
    }
    __syncthreads();
    // terrain base: LDS tile origin (r0-H, oxl), or the global post (r0, c0)
    const int16_t *zb = kLds ? tile : z + r0 * ld + c0;
    const int64_t zb_off = kLds ? 0 : r0 * ld + c0;  // zb's element offset in z (global reads)
    // LDS byte address of the tile
    const int tb = (int)(uint32_t)(uintptr_t)(const __attribute__((address_space(3))) char *)tile;
    const int rs = kLds ? pitch : (int)ld;
    const int tile_rows = (int)((r0 + T > nrows ? nrows : r0 + T) - r0);
    const int tile_cols = (int)((c0 + T > ncols ? ncols : c0 + T) - c0);
    const int R2 = R * R;
    const int nposts = T * T, nbatch = (nposts + 63) >> 6;

    auto claim = [&]() {
        int bt = 0;
        if (lane == 0)
            bt = atomicAdd(&s_batch, 1);
        // wave-uniform: keeps the queue bookkeeping in scalar registers
        return __builtin_amdgcn_readfirstlane(__shfl(bt, 0, 64));
    };
    // this lane's post of batch bt
    auto post_of = [&](int bt, int &py, int &px) {
        const int p = bt * 64 + lane;
        py = p / T;
        px = p - py * T;
        return p < nposts && py < tile_rows && px < tile_cols;
    };

    // ---- the batch being queued: this lane's post and its receiver stream
    int buf = 0, cur_bt = 0;
    bool valid = false;
    uint64_t t = 0;               // post index = stream counter
    int po = 0, Epost = 0;        // post offset from zb, eye elevation
    int bxo = 0, byo = 0;         // clipped box corner relative to the post
    uint32_t wx = 0, wy = 0;      // clipped box extent
    uint32_t tx = 0, ty = 0;      // Lemire thresholds 2^16 mod wx, wy
    uint32_t blk_next = 0;  // next Philox block of the post's stream
    int nbuf = 0;           // words of block blk_next-1 not yet used
    // earlier batches whose tests may still run: bit b of `pending` says
    // that count buffer b holds batch (bt_of >> 16b) & 0xffff
    uint32_t pending = 0;
    uint64_t bt_of = 0;
    // queue of the current chunk: e[j] holds draw j0+j of this lane's post
    // (row j of the wavefront's queue); e[kVixChunk] always holds a no-test
    // word, so that the rows a take may read past the chunk hold no tests
    uint32_t e[kVixChunk + 1];
    e[kVixChunk] = kNoTest;
    int j0 = 0, kc = 0, cursor = 0, total = 0;

    auto setup = [&](int bt) {
        int py, px;
        valid = post_of(bt, py, px);
        const int64_t y = r0 + py, x = c0 + px;
        po = kLds ? (py + H) * pitch + (px + (int)(c0 - oxl)) : py * (int)ld + px;
        Epost = valid ? (int)zb[po] + h_t : 0;
        if (!kLds && valid)
            note(zb_off + po);
        t = (uint64_t)(y * ncols + x);
        const int64_t bx0 = x - R < 0 ? 0 : x - R, bx1 = x + R > ncols - 1 ? ncols - 1 : x + R;
        const int64_t by0 = y - R < 0 ? 0 : y - R, by1 = y + R > nrows - 1 ? nrows - 1 : y + R;
        bxo = (int)(bx0 - x);
        byo = (int)(by0 - y);
        wx = (uint32_t)(bx1 - bx0 + 1);
        wy = (uint32_t)(by1 - by0 + 1);
        tx = 65536u % wx;
        ty = 65536u % wy;
        blk_next = 0;
        nbuf = 0;
        j0 = 0;
    };

    // draws j0 .. j0+kc-1 of every valid lane's post into e[]
    auto generate = [&]() {
        kc = K - j0 < kVixChunk ? K - j0 : kVixChunk;
        const int need = valid ? kc : 0;
        // the queue starts as need empty slots followed by no-test words;
        // every draw (accepted or failed) enters at the end and shifts the
        // queue towards e[0], so the lane still needs draws exactly while
        // e[0] is empty, and after need draws they fill e[kVixChunk-need..]
#pragma unroll
        for (int j = 0; j < kVixChunk; j++)
            e[j] = j < need ? kEmpty : kNoTest;
        // proposals are numbered by slot (wave-uniform: the words left by the
        // previous chunk in slots 0..3, new blocks from slot 4); a lane's
        // live slots run without a gap from its first until its chunk is
        // full, so before slot sl it has rejected sl - s_next proposals in a
        // row, s_next being the slot after its last draw
        int s_next = 4 - nbuf;
        const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
        // one proposal: 16-bit halves scaled to the box with Lemire's
        // rejection, then the disk test; an accepted draw (or a failed one
        // after kVixMaxAttempts rejections) is appended to the lane's queue.
        // Branch-free, so that the queue shifts in place.
        auto propose = [&](uint32_t u, bool live, int sl) {
            const uint32_t mx = __umul24(u & 0xFFFFu, wx), my = __umul24(u >> 16, wy);
            const int dx = bxo + (int)(mx >> 16);
            const int dy = byo + (int)(my >> 16);
            // every test evaluated (no branches around the later ones); the
            // receiver is off the post and in the disk iff 0 < dx^2 + dy^2 <=
            // R^2, i.e. dx^2 + dy^2 - 1 < R^2 as unsigned values (0 wraps)
            const uint32_t d2m1 = (uint32_t)mad_i24(dy, dy, mad_i24(dx, dx, -1));
            const bool ok = ((mx & 0xFFFFu) >= tx) & ((my & 0xFFFFu) >= ty) & (d2m1 < (uint32_t)R2);
            const bool fail = s_next == sl - (kVixMaxAttempts - 1);
            const bool acc = live && (ok || fail);
            s_next = acc ? sl + 1 : s_next;
#pragma unroll
            for (int j = 0; j + 1 < kVixChunk; j++)
                e[j] = acc ? e[j + 1] : e[j];
            e[kVixChunk - 1] = acc ? (ok ? pack_test(dx, dy) : kNoTest) : e[kVixChunk - 1];
            if (kCount && acc && ok)
                tests++;
        };
        // words left in block blk_next-1 by the previous chunk of the post
        if (__any(e[0] == kEmpty && nbuf > 0)) {
            uint32_t o[4];
            philox4x32_10((uint32_t)t, blk_next - 1, (uint32_t)(t >> 32), 0, k0, k1, o);
            const int nb0 = nbuf;
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const bool live = e[0] == kEmpty && i >= 4 - nb0;
                if (K > kVixChunk)  // words left matter only to a later chunk
                    nbuf = live ? 3 - i : nbuf;
                propose(o[i], live, i);
            }
        }
        // a new block per round for every lane that still needs draws (the
        // exit test at the bottom: the queue then stays in its registers
        // across rounds)
        if (__any(e[0] == kEmpty)) {
            int sl = 4;  // slot of the round's first word
            do {
                uint32_t o[4];
                philox4x32_10((uint32_t)t, blk_next, (uint32_t)(t >> 32), 0, k0, k1, o);
                const bool want = e[0] == kEmpty;
                blk_next += want ? 1 : 0;
#pragma unroll
                for (int i = 0; i < 4; i++) {
                    const bool live = e[0] == kEmpty;
                    if (K > kVixChunk)
                        nbuf = live ? 3 - i : nbuf;
                    propose(o[i], live, sl + i);
                }
                sl += 4;
            } while (__any(e[0] == kEmpty));
        }
        // rows 0..kc-1 to e[0..kc-1], no-test words shifted in behind them
        for (int s = kc; s < kVixChunk; s++) {
#pragma unroll
            for (int j = 0; j < kVixChunk; j++)
                e[j] = e[j + 1];
        }
        cursor = 0;
        total = kc * 64;
    };

    // write out the counts of batch bt (held in buffer bf) and clear them
    auto retire = [&](int bf, int bt) {
        int py, px;
        const bool v = post_of(bt, py, px);
        uint32_t *w = &cnt[bf * 16 + (lane >> 2)];
        const uint32_t c = (*w >> ((lane & 3) << 3)) & 0xFFu;
        if (v)
            count[(r0 + py) * ncols + (c0 + px)] = (uint8_t)c;
        *w = 0;  // the four lanes of the word read it above, in wavefront order
    };
    auto add_visible = [&](int cidx) {
        atomicAdd(&cnt[cidx >> 2], 1u << ((cidx & 3) << 3));
    };

    bool more = true;  // further batches may remain in the tile
    const int bt_first = claim();
    // a wavefront that finds no batch left goes straight to the stats below
    const bool have = bt_first < nbatch;
    if (have) {
        cur_bt = bt_first;
        setup(bt_first);
        generate();
    }
    int act = 0;  // this lane runs a test (an int: the ballot below is one compare)
    // LOS state: n major steps, mn minor steps; e = r - n < 0 with r the
    // minor remainder, kept as an unsigned word so that e + mn >= 0 is the
    // carry of the add; off: the current post (its LDS byte address, or its
    // offset in elements from zb); rhs: segment height at the current
    // step (scaled by n); k: steps left; pl: count slot
    int n = 0, mn = 0, off = 0, smaj = 0, smin = 0, rhs = 0, dz = 0, k = 0, pl = 0;
    uint32_t eu = 0;
    // idle lanes take the next tests of the queue, in order
    auto take = [&]() {
        const uint64_t m = __ballot(act == 0);
        // queue position of this lane's test: cursor + idle lanes below it
        const int idx = (int)__builtin_amdgcn_mbcnt_hi(
            (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, (uint32_t)cursor));
        const int src = idx & 63;
        // positions cursor .. cursor+63 hold every lane once: lane L's entry
        // is in row cursor/64 when L >= cursor%64, else in the next row (row
        // indexes wave-uniform; positions from total on hold no tests)
        const int row = cursor >> 6;
        const int row1 = row + 1;
        uint32_t v0 = e[row], v1 = e[row1];  // indexed register reads
        // both rows in registers before the select (else the select moves
        // into the index, which is then per lane and sends e[] to scratch)
        asm volatile("" : "+v"(v0), "+v"(v1));
        const uint32_t mine = lane >= (cursor & 63) ? v0 : v1;
        const uint32_t ent = lane_read(src, mine);
        const int spo = (int)lane_read(src, (uint32_t)po);
        const int sE = (int)lane_read(src, (uint32_t)Epost);
        if (act == 0 && (int)ent < (int)kNoTest) {
            const int dx = (int)ent >> 16, dy = (int)(ent << 16) >> 16;
            // unit steps along x and y (0 along an axis the line does not
            // move on) and the extents |d| = d * sign(d)
            const int ux = sign3(dx), uy = sign3(dy);
            const int adx = mul_i24(dx, ux), ady = mul_i24(dy, uy);
            const bool xmaj = adx >= ady;
            const int cidx = (buf << 6) | src;
            n = xmaj ? adx : ady;
            if (n <= 1) {
                add_visible(cidx);  // adjacent: always visible
            } else {
                const int es = kLds ? 2 : 1;  // offset units per post
                // with a unit step of 0 along an axis the line does not move
                // on, the minor step is 0 when the minor extent is 0, so the
                // second post of a sample (minor offset q+1) is read at offset
                // q, inside the observer-receiver box (its weight r is always 0)
                const int gx = ux * es;
                // in LDS the row step (2 * pitch bytes) is below 2^23; a global
                // row step (ld) may not be
                const int gy = kLds ? mul_i24_s(uy, rs * 2) : (uy < 0 ? -rs : uy > 0 ? rs : 0);
                mn = xmaj ? ady : adx;
                smaj = xmaj ? gx : gy;
                smin = xmaj ? gy : gx;
                off = kLds ? tb + spo * 2 : spo;
                const int tgt = kLds ? mad_i24_s(dy, rs * 2, off) + dx * 2 : spo + dy * rs + dx;
                const int Zt = kLds ? lds_read_i16(tgt) : (int)zb[tgt];
                if (!kLds)
                    note(zb_off + tgt);
                rhs = mul_i24(sE, n);  // |sE| < 2^17, n < 2^14
                dz = Zt + (h_r - sE);
                eu = (uint32_t)-n;
                k = n - 1;  // steps left
                pl = cidx;
                act = 1;
            }
        }
        cursor += (int)__builtin_popcountll(m);
    };

    // kSPI steps of every active test: positions and reads first, then the
    // comparisons, so a test waits for memory once per block
    auto step_block = [&]() {
        if (act == 0)
            return;
        int sa[kSPI], sb[kSPI], se[kSPI];
#pragma unroll
        for (int sp = 0; sp < kSPI; sp++) {
            uint32_t e1;
            const bool wrap = __builtin_add_overflow(eu, (uint32_t)mn, &e1);
            eu = wrap ? e1 - (uint32_t)n : e1;
            off += smaj + (wrap ? smin : 0);
            se[sp] = (int)eu;
            if (kLds) {
                // past the end of the LOS these reads land in the halo
                sa[sp] = lds_read_i16(off);
                sb[sp] = lds_read_i16(off + smin);
            } else {
                sa[sp] = 0;
                sb[sp] = 0;
                if (sp == 0 || sp < k) {
                    // both posts lie in the observer-receiver box: minor
                    // offsets q and q+1 <= |minor| (q+1 = q when |minor| = 0)
                    sa[sp] = zb[off];
                    sb[sp] = zb[off + smin];
                    note(zb_off + off);
                    note(zb_off + off + smin);
                }
            }
        }
        // terrain above the segment: z0*n + (z1-z0)*r = z1*n + (z1-z0)*e
        bool blocked = false;
        int first = kSPI;
#pragma unroll
        for (int sp = 0; sp < kSPI; sp++) {
            rhs += dz;
            const int S = mad_i24(sb[sp] - sa[sp], se[sp], mul_i24(sb[sp], n));
            // k >= 1 at every block start
            const bool bs = (sp == 0 || sp < k) && S > rhs;
            blocked |= bs;
            if (kCount && bs && first == kSPI)
                first = sp;
        }
        if (kCount)
            steps += blocked ? first + 1 : (k < kSPI ? k : kSPI);
        k -= kSPI;
        if (blocked || k <= 0) {
            if (!blocked)
                add_visible(pl);
            act = 0;
        }
    };

    for (; have;) {
        // the hot loop: the queue holds tests
        while (cursor < total) {
            take();
            step_block();
        }
        // queue drained: next chunk of this batch, or the next batch once
        // the count buffer it takes has no test running
        bool gen = false;
        if (j0 + kc < K) {
            j0 += kc;
            gen = true;
        } else if (more) {
            const int nb = (buf + 1) & (kVixBufs - 1);
            bool can = true;
            if (pending & (1u << nb)) {
                if (__any(act != 0 && (pl >> 6) == nb)) {
                    can = false;
                } else {
                    retire(nb, (int)((bt_of >> (16 * nb)) & 0xFFFF));
                    pending &= ~(1u << nb);
                }
            }
            if (can) {
                const int bt = claim();
                if (bt >= nbatch) {
                    more = false;
                } else {
                    pending |= 1u << buf;
                    bt_of = (bt_of & ~(0xFFFFull << (16 * buf))) |
                            ((uint64_t)cur_bt << (16 * buf));
                    buf = nb;
                    cur_bt = bt;
                    setup(bt);
                    gen = true;
                }
            }
        }
        if (gen) {
            generate();
            continue;
        }
        if (!more && !__any(act != 0))
            break;
        // no new tests yet (or none left): advance the running ones
        step_block();
    }
    if (have) {
        retire(buf, cur_bt);
        for (int bf = 0; bf < kVixBufs; bf++)
            if (pending & (1u << bf))
                retire(bf, (int)((bt_of >> (16 * bf)) & 0xFFFF));
    }
    if (kCount) {
        atomicAdd(&stats[0], (unsigned long long)steps);
        atomicAdd(&stats[1], (unsigned long long)tests);
        // offsets as signed values biased by 2^63, so that an unsigned
        // minimum/maximum orders them (a negative offset stays below 0)
        if (rd_lo <= rd_hi) {
            atomicMin(&stats[2], (unsigned long long)rd_lo ^ (1ull << 63));
            atomicMax(&stats[3], (unsigned long long)rd_hi ^ (1ull << 63));
        }
    }
}

__global__ void vix_stats_reset(unsigned long long *stats)
{
    stats[0] = 0;
    stats[1] = 0;
    stats[2] = ~0ull;
    stats[3] = 0;
}

// stats[2..3] back from the biased form; an empty range reads as [0, -1]
__global__ void vix_stats_finish(unsigned long long *stats)
{
    if (stats[2] > stats[3]) {
        stats[2] = 0;
        stats[3] = ~0ull;
    } else {
        stats[2] ^= 1ull << 63;
        stats[3] ^= 1ull << 63;
    }
}

}  // namespace

// Launches the global-read instantiations (large ROI).  They live in a
// translation unit of their own (vix_global.hip) so that they can be compiled
// with another instruction scheduler than the LDS ones here.
void vix_launch_global(bool with_stats, unsigned grid, size_t lds, hipStream_t s,
                       const int16_t *z, int64_t nrows, int64_t ncols, int64_t ld, int R,
                       int h_t, int h_r, int K, uint64_t seed, uint8_t *count, int T,
                       int64_t tiles_r, int64_t tiles_c, int64_t per_xcd, int tile_bytes, int dma,
                       unsigned long long *stats);
}  // namespace siting

#ifndef SITING_VIX_GLOBAL_TU
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
    if (roi > kVixMaxRoi) {
        set_error("%s: roi %d above the supported %d", fn, roi, kVixMaxRoi);
        return SITING_E_UNSUPPORTED;
    }
    // Largest tile side (multiple of 8, <= 128) whose haloed tile (halo: the
    // ROI plus kSPI-1 steps past a line's end) and the count buffers fit in
    // LDS (every instantiation declares the same static LDS).
    const int lds_max = kernel_max_dynamic_lds(reinterpret_cast<const void *>(&vix_kernel<true, false>));
    const int queue_bytes = kVixWaves * kVixWaveLds;
    const int halo = roi + kSPI - 1;
    int T = 0;
    for (int c = 128; c >= 16; c -= 8) {
        int64_t bytes = (((int64_t)(c + 2 * halo) * (c + 2 * halo + 2) * 2 + 15) & ~15ll) + queue_bytes;
        if (bytes <= lds_max) {
            T = c;
            break;
        }
    }
    const bool use_lds = T > 0;
    if (!use_lds)
        T = 64;
    if ((int64_t)(T + 2 * roi + 2) * ld >= ((int64_t)1 << 31)) {
        set_error("%s: roi*ld too large for 32-bit offsets", fn);
        return SITING_E_UNSUPPORTED;
    }
    const int64_t tiles_r = (nrows + T - 1) / T, tiles_c = (ncols + T - 1) / T;
    const int64_t ntiles = tiles_r * tiles_c;
    const int64_t per_xcd = (ntiles + 7) / 8;
    const int64_t grid = per_xcd * 8;
    if (grid > INT32_MAX) {
        set_error("%s: terrain too large", fn);
        return SITING_E_UNSUPPORTED;
    }
    const int tile_bytes = use_lds ? (int)((((int64_t)(T + 2 * halo) * (T + 2 * halo + 2) * 2) + 15) & ~15ll) : 0;
    // direct HBM-to-LDS staging reads whole dwords: rows must start dword-aligned
    // and hold an even number of posts, so that no dword passes a row's end
    const int dma = (ld % 2 == 0) && (ncols % 2 == 0) && ((uintptr_t)z % 4 == 0);
    const size_t lds = (size_t)tile_bytes + queue_bytes;
    hipStream_t s = as_stream(stream);
    if (stats) {
        hipLaunchKernelGGL(vix_stats_reset, dim3(1), dim3(1), 0, s, stats);
        int rc = check_launch("vix_stats_reset");
        if (rc != SITING_OK)
            return rc;
    }
#define VIX_LAUNCH(LDS, CNT)                                                                   \
    hipLaunchKernelGGL((vix_kernel<LDS, CNT>), dim3((unsigned)grid), dim3(kVixThreads), lds, s, \
                       z, nrows, ncols, ld, roi, h_t, h_r, K, seed, count, T, tiles_r, tiles_c,  \
                       per_xcd, tile_bytes, dma, stats)
    if (use_lds && stats)
        VIX_LAUNCH(true, true);
    else if (use_lds)
        VIX_LAUNCH(true, false);
    else
        vix_launch_global(stats != nullptr, (unsigned)grid, lds, s, z, nrows, ncols, ld, roi, h_t,
                          h_r, K, seed, count, T, tiles_r, tiles_c, per_xcd, tile_bytes, dma,
                          stats);
#undef VIX_LAUNCH
    int rc = check_launch("vix_kernel");
    if (rc == SITING_OK && stats) {
        hipLaunchKernelGGL(vix_stats_finish, dim3(1), dim3(1), 0, s, stats);
        rc = check_launch("vix_stats_finish");
    }
    return rc;
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
#endif  // SITING_VIX_GLOBAL_TU
