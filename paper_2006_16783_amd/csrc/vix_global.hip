// VIX: the global-read instantiations of the kernel (ROI too large for an LDS
// tile), compiled from the same source as vix.hip but in a translation unit of
// their own, so that they keep the default instruction scheduler: their lines
// of sight are read through the caches, where the schedule that suits the LDS
// path issues loads less well.
#define SITING_VIX_GLOBAL_TU
#include "vix.hip"

namespace siting {

void vix_launch_global(bool with_stats, unsigned grid, size_t lds, hipStream_t s,
                       const int16_t *z, int64_t nrows, int64_t ncols, int64_t ld, int R,
                       int h_t, int h_r, int K, uint64_t seed, uint8_t *count, int T,
                       int64_t tiles_r, int64_t tiles_c, int64_t per_xcd, int tile_bytes, int dma,
                       unsigned long long *stats)
{
    if (with_stats)
        hipLaunchKernelGGL((vix_kernel<false, true>), dim3(grid), dim3(kVixThreads), lds, s, z,
                           nrows, ncols, ld, R, h_t, h_r, K, seed, count, T, tiles_r, tiles_c,
                           per_xcd, tile_bytes, dma, stats);
    else
        hipLaunchKernelGGL((vix_kernel<false, false>), dim3(grid), dim3(kVixThreads), lds, s, z,
                           nrows, ncols, ld, R, h_t, h_r, K, seed, count, T, tiles_r, tiles_c,
                           per_xcd, tile_bytes, dma, stats);
}

}  // namespace siting
