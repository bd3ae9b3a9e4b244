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

constexpr int32_t kMaxRoi = 16383;
constexpr int32_t kMaxHeight = 32767;

}  // namespace siting
