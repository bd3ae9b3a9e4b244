/*
 * siting.h -- C ABI of libsiting.so, the MI355X (gfx950) implementation of the
 * multiple-observer siting pipeline of Franklin, Magalhaes and Li, "Siting
 * thousands of radio transmitter towers on terrains with billions of points"
 * (arXiv 2006.16783), section "The multiple transmitter siting process":
 *
 *     VIX -> FINDMAX -> VIEWSHED -> SITE
 *
 * plus the learned ranking (a small CNN whose score can replace VIX as the
 * FINDMAX key).
 *
 * Conventions (every entry point):
 *  - Pointers are DEVICE pointers unless the parameter name ends in _host.
 *    The caller owns every buffer; the library never allocates device memory.
 *    Scratch memory is passed in as a workspace whose size a *_workspace_size
 *    query returns.
 *  - Work is enqueued asynchronously on `stream` (a hipStream_t; NULL = the
 *    default stream).  Outputs are valid once the stream has synchronised.
 *  - Return value: SITING_OK (0) or a negative SITING_E_* code.  Arguments are
 *    validated on the host before anything is enqueued; on error nothing is
 *    enqueued and siting_last_error() (thread-local) describes the problem.
 *  - Terrain: int16 elevation posts, row-major, nrows x ncols, leading
 *    dimension ld >= ncols (posts between row starts).  x is the column, y the
 *    row, posts one unit apart (section "Terrain visibility").  All post
 *    indices are int64 (y * ncols + x), since 46400^2 > 2^31.
 *  - Heights h_t (transmitter) and h_r (receiver) are integers in z's unit,
 *    0 <= h <= 32767; the ROI is an integer number of posts, 1 <= roi <= 16383.
 *  - All integer results are deterministic and independent of the schedule.
 */
#ifndef SITING_H
#define SITING_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SITING_ABI_VERSION 1

enum {
    SITING_OK = 0,
    SITING_E_INVALID = -1,      /* bad argument (null pointer, range, shape) */
    SITING_E_UNSUPPORTED = -2,  /* valid but beyond the library's limits */
    SITING_E_HIP = -3,          /* a HIP runtime call failed */
    SITING_E_WORKSPACE = -4,    /* workspace missing or too small */
    SITING_E_INTERNAL = -5      /* internal invariant broken */
};

/* One observer (tentative transmitter) and its viewshed parameters
 * (Definitions: transmitter, transmitter height, radius of interest,
 * receiver height).  Plain 20-byte record, 4-byte aligned. */
typedef struct {
    int32_t x;    /* column of the transmitter base, 0 <= x < ncols */
    int32_t y;    /* row, 0 <= y < nrows */
    int32_t roi;  /* radius of interest in posts, 1..16383 */
    int32_t h_t;  /* transmitter height above its base, 0..32767 */
    int32_t h_r;  /* receiver height above the terrain, 0..32767 */
} siting_observer;

/* Launch schedule of siting_viewshed_batch (see that function). */
typedef struct {
    int32_t waves;          /* wavefronts (64 lanes) per workgroup: 1..16 */
    int32_t groups_per_cu;  /* resident workgroups per compute unit: 1..16 */
    int32_t stage_rmax;     /* observers with roi <= stage_rmax stage their
                               terrain in LDS (one half-window at a time);
                               larger ones read the terrain through the cache
                               hierarchy. 0 = none */
    int32_t ray_per_wave;   /* 0: one ray per lane; 1: one wavefront per ray
                               (64 samples of the ray at a time, the horizon
                               as an exact prefix maximum across lanes), for
                               the observers whose terrain is read from global
                               memory (not staged); same bits either way */
} siting_schedule;

enum { SITING_KEY_U8 = 0, SITING_KEY_F32 = 1 };
enum { SITING_SINK_BITMAP = 0, SITING_SINK_COUNT = 1 };

int siting_abi_version(void);

/* Description of the last error on the calling thread ("" if none). */
const char *siting_last_error(void);

/* Number of compute units of the current device (for sizing schedules). */
int siting_device_cus(int32_t *cus_host);

/* ---------------------------------------------------------------- VIX ----
 * Estimated visibility index of every post (stage Vix): for each post T and
 * each of K draws, a receiver P uniform over the lattice cells of T's ROI disk
 * that lie inside the terrain (P != T), and the line-of-sight test between
 * the eye z[T]+h_t and the receiver top z[P]+h_r.  The LOS samples the
 * terrain where the segment crosses each grid line of its major axis,
 * linearly interpolated between the two adjacent posts ("Terrain
 * visibility"), and is blocked only if the terrain is strictly above the
 * segment.
 * Post t = y*ncols+x owns one stream of 32-bit words: word a is word a%4 of
 * Philox4x32-10(counter {t mod 2^32, a/4, t / 2^32, 0},
 * key {seed mod 2^32, seed / 2^32}).  Each word u proposes one receiver in
 * the terrain-clipped box [bx0, bx0+wx) x [by0, by0+wy) around T: with
 * mx = (u & 0xffff) * wx and my = (u >> 16) * wy (Lemire's multiply-shift),
 * the proposal is rejected if (mx & 0xffff) < 2^16 mod wx or
 * (my & 0xffff) < 2^16 mod wy, else P = (bx0 + (mx >> 16), by0 + (my >> 16))
 * (exactly uniform over the box); it is accepted iff also P != T and
 * |P-T|^2 <= roi^2.  Draw j is the next accepted proposal of the stream;
 * after 64 consecutive rejections the draw fails (counts as not visible)
 * and draw j+1 continues with the next word.
 *   z      : terrain (device), nrows x ncols, leading dimension ld
 *   nrows, ncols >= 2; K in 1..255
 *   count  : out (device), nrows x ncols uint8, contiguous row-major: the
 *            number of visible receivers of each post (0..K).  */
int siting_vix(const int16_t *z, int64_t nrows, int64_t ncols, int64_t ld,
               int32_t roi, int32_t h_t, int32_t h_r, int32_t K, uint64_t seed,
               uint8_t *count, void *stream);

/* The same computation as siting_vix (identical count output), in a
 * counting variant for measurement: stats (device, uint64[4]) receives
 *   [0] the number of line-of-sight steps executed (grid-line samples
 *       tested, up to and including the first blocking one),
 *   [1] the number of line-of-sight tests,
 *   [2], [3] the lowest and highest element offset from z (as int64) of any
 *       terrain post the kernel reads from global memory, staging included
 *       ([0, -1] if it reads none); every read lies in the terrain, i.e.
 *       0 <= [2] and [3] <= (nrows-1)*ld + ncols-1.
 * Slower than siting_vix; not meant for production runs. */
int siting_vix_stats(const int16_t *z, int64_t nrows, int64_t ncols, int64_t ld,
                     int32_t roi, int32_t h_t, int32_t h_r, int32_t K, uint64_t seed,
                     uint8_t *count, uint64_t *stats, void *stream);

/* ------------------------------------------------------------ FINDMAX ----
 * Spatially spread candidates (stage Findmax): the terrain is split into a
 * grid_r x grid_c grid of blocks, block (bi,bj) spanning rows
 * [floor(bi*nrows/grid_r), floor((bi+1)*nrows/grid_r)) and likewise columns;
 * each block keeps its k best posts.
 *   key_type SITING_KEY_U8 : key is uint8[nrows*ncols] (a VIX count); rank by
 *            (key desc, z desc, linear index asc); key_stride must be 1.
 *   key_type SITING_KEY_F32: key is float[ceil(nrows/s) * ceil(ncols/s)],
 *            s = key_stride >= 1, one score per s x s cell; a cell belongs
 *            to the block holding its corner post (i*s, j*s); rank by (key
 *            desc, cell index asc), NaN as -infinity; a winning cell is
 *            returned as its highest post (elevation desc, index asc), the
 *            post siting_cnn_score_terrain scores.
 *   cand   : out (device), int64[grid_r*grid_c*k]: blocks in row-major
 *            order, each with k post indices best first, padded with -1.
 *   1 <= grid_r <= nrows, 1 <= grid_c <= ncols, 1 <= k <= 32.
 * The paper's own default is blocks of width ROI/3 and k = 20, i.e.
 * grid = round(N / floor(ROI/3)) per side. */
int siting_findmax(const void *key, int32_t key_type, int32_t key_stride,
                   const int16_t *z, int64_t nrows, int64_t ncols, int64_t ld,
                   int32_t grid_r, int32_t grid_c, int32_t k, int64_t *cand,
                   void *stream);

/* ----------------------------------------------------------- VIEWSHED ----
 * Window bitmaps (stage Viewshed; bitmaps in 64-bit words).  Observer i's
 * window covers rows [max(0,y-R), min(nrows-1,y+R)] and the 64-bit words
 * [max(0,x-R)>>6, min(ncols-1,x+R)>>6] of each row, stored row-major at
 * bitmaps + offsets[i]; bit (c & 63) of word (c >> 6) is column c, exactly
 * as in a full-terrain bitmap of ceil(ncols/64) words per row.  Bits outside
 * the ROI disk, outside the terrain, or in padding are 0.
 *
 * Host-only.  Writes offsets_host[0..n] (offsets_host[n] = total words) and
 * returns the total number of words, or a negative SITING_E_* code. */
int64_t siting_viewshed_layout(const siting_observer *obs_host, int64_t n, int64_t nrows,
                               int64_t ncols, int64_t *offsets_host);

/* Host-only.  A processing order (permutation of 0..n-1) by decreasing
 * cost (roi, then index), so that a persistent launch takes the longest
 * observers first.  Returns SITING_OK or an error code. */
int siting_viewshed_order(const siting_observer *obs_host, int64_t n, int32_t *order_host);

/* Workspace bytes of siting_viewshed_batch (a work-queue counter and an
 * error word). */
size_t siting_viewshed_workspace_size(void);

/* The default schedule for observers with ROI up to rmax. */
int siting_viewshed_default_schedule(int32_t rmax, siting_schedule *sched_host);

/* Viewsheds of n observers in one persistent launch.  Per observer: rays
 * from the observer to every boundary cell of its terrain-clipped
 * (2R+1)^2 window; along each ray, at major-axis step k (k*|minor| =
 * q*n + r) the terrain sample is S_k = z0*(n-r) + z1*r (n times the linear
 * interpolation between the posts at minor offsets q and q+1), the marked
 * cell is the one at minor offset q + [2r >= n] (nearest, ties away from the
 * observer), and the ray stops when that cell leaves the ROI disk.  With the
 * horizon (S_J, J) the cell is visible iff
 *     (S_k + h_r*n - E*n) * J >= (S_J - E*n) * k,    E = z[obs] + h_t,
 * and the horizon moves to (S_k, k) iff (S_k - E*n)*J > (S_J - E*n)*k; the
 * first step has no horizon and is visible.  The observer's own cell is
 * visible.  The viewshed is the OR over rays.  All comparisons are exact
 * integer arithmetic (stage Viewshed: walk each line of sight updating a
 * horizon angle).
 *   obs     : device array of n observers
 *   offsets : device int64[n+1] from siting_viewshed_layout
 *   order   : device int32[n] processing order, or NULL for 0..n-1
 *   sched_host : schedule, or NULL for siting_viewshed_default_schedule(max roi)
 *   sink SITING_SINK_BITMAP: bitmaps (device uint64[offsets[n]]) is written;
 *        visible/cells may be NULL.
 *   sink SITING_SINK_COUNT : visible[i] = number of visible cells (including
 *        the observer), cells[i] = number of ROI-disk cells inside the
 *        terrain (the visibility index is visible/cells, Definitions);
 *        bitmaps and offsets may be NULL when rmax <= 1087.
 *   rmax    : an upper bound of every observer's roi (sizes LDS).  The
 *        observer records are not read by the host: a record with roi > rmax
 *        or any field out of range is skipped (its bitmap words are left
 *        untouched; sink COUNT writes 0 and 0).  A whole-window bitmap fits
 *        LDS up to rmax 543; above that every observer is swept one
 *        quadrant at a time from global memory (the schedule's stage_rmax is
 *        then ignored), up to rmax 1087; above that each observer's window is
 *        cleared in `bitmaps` and marked there with atomic ORs (same bits),
 *        so `bitmaps` and `offsets` are required with either sink (sink
 *        COUNT uses them as scratch and leaves the windows there).
 *   ws, ws_bytes : workspace of siting_viewshed_workspace_size() bytes. */
int siting_viewshed_batch(const int16_t *z, int64_t nrows, int64_t ncols, int64_t ld,
                          const siting_observer *obs, int64_t n, const int64_t *offsets,
                          const int32_t *order, int32_t rmax,
                          const siting_schedule *sched_host, int32_t sink,
                          uint64_t *bitmaps, uint32_t *visible, uint32_t *cells,
                          void *ws, size_t ws_bytes, void *stream);

/* Exact visibility index of n observers from the counts of sink
 * SITING_SINK_COUNT (Definitions: the fraction of the receivers within the
 * ROI that are visible; the observer's own cell is not a receiver):
 *     vi[i] = (visible[i] - 1) / (cells[i] - 1)
 * as the correctly rounded float32 quotient of the two counts converted to
 * float32 (exact conversions up to 2^24, i.e. every ROI <= 2310), and 0 when
 * visible[i] = 0 or cells[i] <= 1 (a skipped record).
 *   visible, cells : device uint32[n];  vi : out, device float[n]. */
int siting_visibility_index(const uint32_t *visible, const uint32_t *cells, int64_t n,
                            float *vi, void *stream);

/* Exact per-cell viewsheds, for measuring the sweep above against exact line
 * of sight (the R3 family the paper cites as prior art; O(R^3) per observer,
 * not part of the siting path): every lattice cell P of the ROI disk inside
 * the terrain is visible iff the line of sight between the eye z[obs]+h_t
 * and the receiver top z[P]+h_r is clear, by the test siting_vix describes;
 * the observer's own cell is visible.  Same window layout and bitmaps as
 * siting_viewshed_batch (offsets from siting_viewshed_layout; bitmaps device
 * uint64[offsets[n]]); a record with a field out of range is skipped (its
 * words are left untouched). */
int siting_viewshed_r3(const int16_t *z, int64_t nrows, int64_t ncols, int64_t ld,
                       const siting_observer *obs, int64_t n, const int64_t *offsets,
                       uint64_t *bitmaps, void *stream);

/* Times the candidate schedules of siting_viewshed_batch on the given
 * observers (synchronising the stream) and writes the fastest to
 * best_host; every candidate produces the same bits.  times_ms_host (may be
 * NULL) receives up to max_times timings in the order of
 * siting_autotune_candidates.  bitmaps must hold offsets[n] words. */
int siting_autotune(const int16_t *z, int64_t nrows, int64_t ncols, int64_t ld,
                    const siting_observer *obs, int64_t n, const int64_t *offsets,
                    const int32_t *order, int32_t rmax, uint64_t *bitmaps, void *ws,
                    size_t ws_bytes, void *stream, siting_schedule *best_host,
                    float *times_ms_host, int32_t max_times);

/* Host-only: the candidate schedules the autotuner tries for rmax. */
int siting_autotune_candidates(int32_t rmax, siting_schedule *out_host, int32_t max_out);

/* --------------------------------------------------------------- SITE ----
 * Greedy observer selection (stage Site): starting from an empty cumulative
 * viewshed C, repeatedly take the candidate with the largest gain
 * |V_i \ C| (ties to the smallest candidate index), record it and set
 * C |= V_i; stop after max_obs observers, once |C| >= target_cells, or
 * when the best gain is 0.  Evaluated lazily with the stage's stated bound
 * (a gain can only shrink as C grows, so a stale gain is an upper bound):
 * the top candidate is taken only once its gain is fresh, which makes the
 * selection exactly the plain greedy one; a stale top is re-evaluated and
 * taken at once if it still beats every other key.  One wavefront runs the
 * rounds; when some window exceeds 1024 words, three more join the rounds
 * whose window does (the selection is the same either way).
 *   bitmaps/offsets/obs : as produced by siting_viewshed_batch (device)
 *   n: 1 .. 4,194,304 (the maxima of the keys over blocks of 512 candidates,
 *   12 bytes per block, live in LDS; SITING_E_UNSUPPORTED beyond); windows must be
 *   those of the same nrows x ncols terrain; a record with a position or roi
 *   out of range counts as gaining nothing
 *   cumulative : out (device) uint64[nrows * ceil(ncols/64)], overwritten
 *   selected, gains : out (device) int64[max_obs]; entries past *nselected
 *                     are left untouched
 *   nselected  : out (device) int32, number selected
 *   ws, ws_bytes : workspace of siting_greedy_workspace_size(n) bytes (the
 *                  size serves siting_greedy_intervisible as well) */
size_t siting_greedy_workspace_size(int64_t n);
int siting_greedy(const uint64_t *bitmaps, const int64_t *offsets, const siting_observer *obs,
                  int64_t n, int64_t nrows, int64_t ncols, int32_t max_obs, int64_t target_cells,
                  uint64_t *cumulative, int64_t *selected, int64_t *gains, int32_t *nselected,
                  void *ws, size_t ws_bytes, void *stream);

/* The same selection under intervisibility, a constraint the paper names
 * among the variants of the problem (transmitters required to be visible from
 * other transmitters): the first pick is free; after it, a candidate competes
 * only if its own post lies in the cumulative viewshed C, i.e. it is visible
 * (as a receiver, h_r above the terrain) from at least one transmitter already
 * chosen, so every transmitter after the first is seen by an earlier one.  A
 * round takes the competing candidate with the largest gain (ties to the
 * smallest index); the run also stops when no competing candidate gains
 * anything.  A record with a position or roi out of range never competes
 * after the first round.  Arguments, outputs and errors as siting_greedy;
 * ws, ws_bytes: siting_greedy_workspace_size(n) bytes. */
int siting_greedy_intervisible(const uint64_t *bitmaps, const int64_t *offsets,
                               const siting_observer *obs, int64_t n, int64_t nrows,
                               int64_t ncols, int32_t max_obs, int64_t target_cells,
                               uint64_t *cumulative, int64_t *selected, int64_t *gains,
                               int32_t *nselected, void *ws, size_t ws_bytes, void *stream);

/* The same selection as siting_greedy for large windows, each round spread
 * over the GPU: up to `batch` stale top candidates (the top candidate of the
 * top block and of the blocks whose maxima carry the largest gain bounds) are
 * re-evaluated by one workgroup each, then the largest key overall is taken
 * if it is fresh (the stage's bound makes that the plain greedy choice).
 * Rounds are enqueued by the host in batches and the call SYNCHRONIZES
 * `stream` (it returns when the selection is complete).  Arguments, outputs
 * and errors as siting_greedy; 1 <= batch <= 1024; ws, ws_bytes:
 * siting_greedy_workspace_size(n) bytes.  Meant for windows of thousands of
 * words (ROI in the hundreds and more), where one workgroup per round is
 * bound by its own memory latency. */
int siting_greedy_parallel(const uint64_t *bitmaps, const int64_t *offsets,
                           const siting_observer *obs, int64_t n, int64_t nrows, int64_t ncols,
                           int32_t max_obs, int64_t target_cells, int32_t batch,
                           uint64_t *cumulative, int64_t *selected, int64_t *gains,
                           int32_t *nselected, void *ws, size_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * selection as siting_greedy, identical outputs, without a workspace
 * argument.  Its state lives in a static device array the library holds on
 * each device until the process ends, sized for up to
 * SITING_GREEDY_NOALLOC_MAX_N candidates (about 12.6 MB); n above that
 * returns SITING_E_UNSUPPORTED.  The call allocates nothing (no hipMalloc,
 * no library allocation).  Every call on one device shares that device's
 * array, which keeps the last call's contents (each call rewrites what it
 * reads, so nothing needs clearing): calls that overlap on one device, on
 * any streams, race and must be serialised by the caller. */
#define SITING_GREEDY_NOALLOC_MAX_N 1048576
int siting_greedy_noalloc(const uint64_t *bitmaps, const int64_t *offsets,
                          const siting_observer *obs, int64_t n, int64_t nrows, int64_t ncols,
                          int32_t max_obs, int64_t target_cells, uint64_t *cumulative,
                          int64_t *selected, int64_t *gains, int32_t *nselected, void *stream);

/* ------------------------------------------------------ LEARNED RANKING ----
 * A small CNN predicting a post's visibility index (Definitions: the visible
 * fraction of the ROI receivers) from the 64 x 64 patch around it, used only
 * as an alternative FINDMAX key (SITING_KEY_F32); VIEWSHED and SITE stay
 * exact.  Not part of the paper's method.
 *   input  P[dy][dx] = bf16(float(z[clamp(cy+dy-32, cx+dx-32)] - z[cy][cx]) * 2^-8)
 *   conv1 4x4 stride 4, 1->16, ReLU (bf16) -> conv2 3x3 stride 2, 16->16, ReLU
 *   (bf16) -> conv3 3x3 stride 2, 16->32, ReLU -> mean over 3x3 -> FC 32->1
 *   -> sigmoid.
 * Convolutions run on BF16 MFMA with FP32 accumulation.  Parameters are one
 * fp32 vector of siting_cnn_param_count() values in the order w1[16][4][4],
 * b1[16], w2[16][3][3][16], b2[16], w3[32][3][3][16], b3[32], wfc[32], bfc.
 * Posts outside the terrain take the nearest edge post. */
int siting_cnn_param_count(void);

/* Workspace bytes for a training batch of `batch` posts (activations kept
 * between siting_cnn_forward and siting_cnn_backward); 0 if batch < 1. */
size_t siting_cnn_workspace_size(int64_t batch);

/* Training forward pass over the posts centres[0..B) (device int64 linear
 * indices).  pred (device float[B], may be NULL) receives the predictions;
 * the activations stay in ws for siting_cnn_backward. */
int siting_cnn_forward(const float *params, const int16_t *z, int64_t nrows, int64_t ncols,
                       int64_t ld, const int64_t *centres, int64_t B, float *pred, void *ws,
                       size_t ws_bytes, void *stream);

/* Gradient of the mean squared error between the predictions of the last
 * siting_cnn_forward on the same ws and labels[0..B) (device float), written
 * to grad (device float[param_count]); loss (device float, may be NULL)
 * receives the loss.  Upstream gradients are rounded to bf16 where they
 * enter an MFMA; every reduction runs in a fixed order (deterministic). */
int siting_cnn_backward(const float *params, const float *labels, int64_t B, float *grad,
                        float *loss, void *ws, size_t ws_bytes, void *stream);

/* One Adam step (Kingma & Ba, bias-corrected; step >= 1) on n fp32 values:
 * params, first and second moments m, v updated in place. */
int siting_cnn_adam(float *params, float *m, float *v, const float *grad, int64_t n,
                    int32_t step, float lr, float beta1, float beta2, float eps, void *stream);

/* Predicted visibility index of every stride x stride cell of the terrain,
 * evaluated at the cell's highest post (elevation desc, index asc; the post
 * a SITING_KEY_F32 FINDMAX returns for the cell): score (device float) has
 * ceil(nrows/stride) x ceil(ncols/stride) entries, row-major.
 * 1 <= stride <= 64. */
int siting_cnn_score_terrain(const float *params, const int16_t *z, int64_t nrows,
                             int64_t ncols, int64_t ld, int32_t stride, float *score,
                             void *stream);

#ifdef __cplusplus
}
#endif
#endif /* SITING_H */
