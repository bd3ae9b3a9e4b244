// Exact visibility index of each observer from the viewshed count sink
// (Definitions: the fraction of the receivers within the ROI that are
// visible; the observer's own cell is neither counted nor a receiver).
#include "common.hpp"

namespace siting {
namespace {

__global__ void visibility_index_kernel(const uint32_t *__restrict__ visible,
                                        const uint32_t *__restrict__ cells, int64_t n,
                                        float *__restrict__ vi)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const uint32_t v = visible[i], c = cells[i];
    // correctly rounded float32 quotient of the two counts (exact as floats
    // up to 2^24, i.e. every disk of ROI <= 2310)
    vi[i] = (v >= 1 && c >= 2) ? __fdiv_rn((float)(v - 1), (float)(c - 1)) : 0.0f;
}

}  // namespace
}  // namespace siting

using namespace siting;

extern "C" int siting_visibility_index(const uint32_t *visible, const uint32_t *cells, int64_t n,
                                       float *vi, void *stream)
{
    clear_error();
    SITING_REQUIRE(n >= 0, "siting_visibility_index: n < 0");
    if (n == 0)
        return SITING_OK;
    SITING_REQUIRE(visible && cells && vi, "siting_visibility_index: NULL pointer");
    const int threads = 256;
    const int64_t blocks = (n + threads - 1) / threads;
    SITING_REQUIRE(blocks <= INT32_MAX, "siting_visibility_index: n too large");
    hipLaunchKernelGGL(visibility_index_kernel, dim3((unsigned)blocks), dim3(threads), 0,
                       as_stream(stream), visible, cells, n, vi);
    return check_launch("visibility_index_kernel");
}
