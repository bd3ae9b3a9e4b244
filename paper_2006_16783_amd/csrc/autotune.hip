// Autotuner of the persistent viewshed launch: times the candidate schedules
// (workgroup size, resident workgroups per CU, LDS staging of the terrain
// quadrant or reads through the cache hierarchy) on the caller's observers and
// keeps the fastest.  Every schedule computes the same bits; only speed
// differs.
#include <algorithm>
#include <vector>

#include "common.hpp"

namespace siting {
int viewshed_launch(const int16_t *z, int64_t nrows, int64_t ncols, int64_t ld,
                    const siting_observer *obs, int64_t n, const int64_t *offsets,
                    const int32_t *order, int32_t rmax, const siting_schedule &sc, int32_t sink,
                    uint64_t *bitmaps, uint32_t *visible, uint32_t *cells, void *ws,
                    hipStream_t s);
int viewshed_lds_bytes(int32_t rmax, int32_t stage_rmax);
int viewshed_max_dynamic_lds();
bool quad_mode(int rmax);
int viewshed_mode(int rmax);
int validate_schedule(const siting_schedule &sc, const char *fn);
}  // namespace siting

using namespace siting;

extern "C" int siting_autotune_candidates(int32_t rmax, siting_schedule *out_host, int32_t max_out)
{
    clear_error();
    SITING_REQUIRE(rmax >= 1 && rmax <= kMaxRoi, "siting_autotune_candidates: bad rmax");
    SITING_REQUIRE(max_out >= 0 && (max_out == 0 || out_host), "siting_autotune_candidates: bad output");
    const int budget = std::min(160 * 1024, viewshed_max_dynamic_lds());
    std::vector<siting_schedule> c;
    // stage everything, nothing, or only the observers up to a partial ROI
    // (uneven batches: small observers from LDS, large ones through L2)
    // (windows too large for an LDS bitmap: quadrant mode, no staging)
    const bool quad = quad_mode(rmax);
    if (viewshed_mode(rmax) == 2) {
        // global-bitmap mode uses no LDS: wavefronts per workgroup and
        // workgroups per CU only
        for (int waves : {8, 16})
            for (int g : {1, 2, 4})
                c.push_back(siting_schedule{waves, g, 0, 0});
    }
    std::vector<int> stages;
    if (viewshed_mode(rmax) != 2)
        stages.push_back(quad ? 0 : rmax);
    if (!quad) {
        stages.push_back(0);
        for (int st : {64, 100, 128, 160, 200, 256})
            if (st < rmax)
                stages.push_back(st);
    }
    for (int stage : stages) {
        int lds = viewshed_lds_bytes(rmax, stage);
        if (lds > budget)
            continue;
        int fit = std::max(1, std::min(16, budget / lds));
        for (int waves : {2, 4, 8, 16}) {
            // quadrant mode sweeps about 2R rays per quadrant: 8 or 16
            // wavefronts; otherwise 2 to 8, and 16 where one workgroup fills
            // the CU's LDS
            if (quad ? waves < 8 : (waves > 8 && fit > 1))
                continue;
            for (int g : {fit, std::max(1, fit / 2)}) {
                siting_schedule s{waves, g, stage, 0};
                bool dup = false;
                for (auto &e : c)
                    dup |= e.waves == s.waves && e.groups_per_cu == s.groups_per_cu &&
                           e.stage_rmax == s.stage_rmax && e.ray_per_wave == s.ray_per_wave;
                if (!dup)
                    c.push_back(s);
            }
        }
    }
    // where observers read their terrain from global memory (staging below
    // rmax), the same schedule with one wavefront per ray as well
    const size_t nlane = c.size();
    for (size_t e = 0; e < nlane; e++)
        if (c[e].stage_rmax < rmax && c[e].waves >= 4) {
            siting_schedule w = c[e];
            w.ray_per_wave = 1;
            c.push_back(w);
        }
    int m = std::min<int>((int)c.size(), max_out);
    for (int i = 0; i < m; i++)
        out_host[i] = c[i];
    return (int)c.size();
}

extern "C" int siting_autotune(const int16_t *z, int64_t nrows, int64_t ncols, int64_t ld,
                               const siting_observer *obs, int64_t n, const int64_t *offsets,
                               const int32_t *order, int32_t rmax, uint64_t *bitmaps, void *ws,
                               size_t ws_bytes, void *stream, siting_schedule *best_host,
                               float *times_ms_host, int32_t max_times)
{
    clear_error();
    const char *fn = "siting_autotune";
    SITING_REQUIRE(best_host != nullptr, "%s: NULL best_host", fn);
    SITING_REQUIRE(n >= 1 && n <= INT32_MAX, "%s: n out of range", fn);
    SITING_REQUIRE(z && obs && offsets && bitmaps, "%s: NULL device pointer", fn);
    SITING_REQUIRE(rmax >= 1 && rmax <= kMaxRoi, "%s: bad rmax", fn);
    SITING_REQUIRE(ld >= ncols && nrows >= 1 && ncols >= 1, "%s: bad terrain shape", fn);
    if (ws == nullptr || ws_bytes < 256) {
        set_error("%s: workspace too small", fn);
        return SITING_E_WORKSPACE;
    }
    siting_schedule cand[128];
    int nc = siting_autotune_candidates(rmax, cand, 128);
    if (nc <= 0) {
        set_error("%s: no schedule fits rmax %d", fn, rmax);
        return SITING_E_UNSUPPORTED;
    }
    nc = std::min(nc, 128);
    hipStream_t s = as_stream(stream);
    hipEvent_t e0, e1;
    SITING_HIP(hipEventCreate(&e0));
    SITING_HIP(hipEventCreate(&e1));
    float best = 1e30f;
    int rc = SITING_OK;
    for (int c = 0; c < nc && rc == SITING_OK; c++) {
        // one warm-up, then the median-free minimum of 3 timed runs
        float tmin = 1e30f;
        for (int rep = 0; rep < 4 && rc == SITING_OK; rep++) {
            if (hipEventRecord(e0, s) != hipSuccess) { rc = SITING_E_HIP; break; }
            rc = viewshed_launch(z, nrows, ncols, ld, obs, n, offsets, order, rmax, cand[c],
                                 SITING_SINK_BITMAP, bitmaps, nullptr, nullptr, ws, s);
            if (rc != SITING_OK)
                break;
            if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
                rc = SITING_E_HIP;
                break;
            }
            float ms = 0;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (rep > 0)
                tmin = std::min(tmin, ms);
        }
        if (rc != SITING_OK)
            break;
        if (times_ms_host && c < max_times)
            times_ms_host[c] = tmin;
        if (tmin < best) {
            best = tmin;
            *best_host = cand[c];
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc == SITING_E_HIP)
        set_error("%s: HIP event failure", fn);
    return rc;
}
