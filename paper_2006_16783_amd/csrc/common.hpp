// Shared host/device plumbing of libsiting: error reporting, launch checks,
// device properties.  Kernels live in the per-stage .hip files.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/siting.h"

namespace siting {

// Thread-local last-error text (siting_last_error).
void set_error(const char *fmt, ...);
void clear_error();

// Return code helpers: validate on the host before any launch.
#define SITING_REQUIRE(cond, ...)                 \
    do {                                          \
        if (!(cond)) {                            \
            ::siting::set_error(__VA_ARGS__);     \
            return SITING_E_INVALID;              \
        }                                         \
    } while (0)

#define SITING_HIP(call)                                                          \
    do {                                                                          \
        hipError_t e_ = (call);                                                   \
        if (e_ != hipSuccess) {                                                   \
            ::siting::set_error("%s failed: %s", #call, hipGetErrorString(e_));  \
            return SITING_E_HIP;                                                  \
        }                                                                         \
    } while (0)

// Checks the launch that was just enqueued.
int check_launch(const char *what);

// Compute units and maximum LDS bytes per workgroup of the current device.
int device_cus();
int device_max_lds();
// Dynamic LDS bytes a launch of `kernel` may request: the device maximum less
// the kernel's static __shared__ variables (the two together must fit, and
// the runtime does not reject a launch that exceeds it).
int kernel_max_dynamic_lds(const void *kernel);

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// Wavefront reductions on DPP lane moves (row shifts by 1, 2, 4, 8, then the
// row broadcasts of lanes 15 and 31): lane 63 ends with the result, which is
// returned to every lane.  Lanes a move leaves without a source, and rows the
// row mask excludes, read the identity 0.
template <int kCtrl, int kRowMask>
__device__ __forceinline__ uint32_t dpp_move(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kCtrl, kRowMask, 0xF, false);
}
template <int kCtrl, int kRowMask>
__device__ __forceinline__ uint64_t dpp_move64(uint64_t v)
{
    return ((uint64_t)dpp_move<kCtrl, kRowMask>((uint32_t)(v >> 32)) << 32) |
           dpp_move<kCtrl, kRowMask>((uint32_t)v);
}
__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v)
{
    uint64_t w;
    w = dpp_move64<0x111, 0xF>(v); v = w > v ? w : v;
    w = dpp_move64<0x112, 0xF>(v); v = w > v ? w : v;
    w = dpp_move64<0x114, 0xF>(v); v = w > v ? w : v;
    w = dpp_move64<0x118, 0xF>(v); v = w > v ? w : v;
    w = dpp_move64<0x142, 0xA>(v); v = w > v ? w : v;
    w = dpp_move64<0x143, 0xC>(v); v = w > v ? w : v;
    return ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), 63) << 32) |
           (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, 63);
}
// sum of 32-bit values (the total must fit 32 bits)
__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v)
{
    v += dpp_move<0x111, 0xF>(v);
    v += dpp_move<0x112, 0xF>(v);
    v += dpp_move<0x114, 0xF>(v);
    v += dpp_move<0x118, 0xF>(v);
    v += dpp_move<0x142, 0xA>(v);
    v += dpp_move<0x143, 0xC>(v);
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

constexpr int32_t kMaxRoi = 16383;
constexpr int32_t kMaxHeight = 32767;

}  // namespace siting
