// Host-side entry points of libsiting: version, error text, device queries,
// and the viewshed layout/order helpers (pure host code).
#include <algorithm>
#include <mutex>
#include <numeric>
#include <vector>

#include "common.hpp"

namespace siting {

static thread_local std::string g_last_error;

void set_error(const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
}

void clear_error() { g_last_error.clear(); }

int check_launch(const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error("launch of %s failed: %s", what, hipGetErrorString(e));
        return SITING_E_HIP;
    }
    return SITING_OK;
}

namespace {
struct DevProps {
    int cus = 0;
    int lds = 0;
};
std::mutex g_props_mu;
DevProps g_props[64];
}  // namespace

static DevProps props()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        return DevProps{};
    std::lock_guard<std::mutex> lk(g_props_mu);
    DevProps &p = g_props[dev];
    if (p.cus == 0) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess)
            p.cus = v;
        v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess)
            p.lds = v;
    }
    return p;
}

int device_cus()
{
    int c = props().cus;
    return c > 0 ? c : 256;
}

int device_max_lds()
{
    int l = props().lds;
    return l > 0 ? l : 160 * 1024;  // gfx950 without a device to ask (host-only use)
}

int kernel_max_dynamic_lds(const void *kernel)
{
    static std::mutex mu;
    static std::vector<std::pair<const void *, int>> cache;
    int stat = -1;
    {
        std::lock_guard<std::mutex> lk(mu);
        for (auto &e : cache)
            if (e.first == kernel)
                stat = e.second;
    }
    if (stat < 0) {
        hipFuncAttributes a{};
        if (hipFuncGetAttributes(&a, kernel) == hipSuccess) {
            stat = (int)a.sharedSizeBytes;
            std::lock_guard<std::mutex> lk(mu);
            cache.emplace_back(kernel, stat);
        } else {
            (void)hipGetLastError();
            stat = 1024;  // no device to ask: a conservative reserve
        }
    }
    return device_max_lds() - ((stat + 15) & ~15);
}

}  // namespace siting

using namespace siting;

extern "C" int siting_abi_version(void) { return SITING_ABI_VERSION; }

extern "C" const char *siting_last_error(void) { return g_last_error.c_str(); }

extern "C" int siting_device_cus(int32_t *cus_host)
{
    SITING_REQUIRE(cus_host != nullptr, "siting_device_cus: cus_host is NULL");
    int dev = 0;
    SITING_HIP(hipGetDevice(&dev));
    *cus_host = device_cus();
    return SITING_OK;
}

static int validate_observers_host(const siting_observer *obs, int64_t n, int64_t nrows,
                                   int64_t ncols, const char *fn)
{
    for (int64_t i = 0; i < n; i++) {
        const siting_observer &o = obs[i];
        if (o.x < 0 || o.x >= ncols || o.y < 0 || o.y >= nrows) {
            set_error("%s: observer %lld at (%d,%d) lies outside the %lldx%lld terrain", fn,
                      (long long)i, o.x, o.y, (long long)nrows, (long long)ncols);
            return SITING_E_INVALID;
        }
        if (o.roi < 1 || o.roi > kMaxRoi) {
            set_error("%s: observer %lld has roi %d outside 1..%d", fn, (long long)i, o.roi,
                      kMaxRoi);
            return SITING_E_INVALID;
        }
        if (o.h_t < 0 || o.h_t > kMaxHeight || o.h_r < 0 || o.h_r > kMaxHeight) {
            set_error("%s: observer %lld has heights (%d,%d) outside 0..%d", fn, (long long)i,
                      o.h_t, o.h_r, kMaxHeight);
            return SITING_E_INVALID;
        }
    }
    return SITING_OK;
}

extern "C" int64_t siting_viewshed_layout(const siting_observer *obs_host, int64_t n,
                                          int64_t nrows, int64_t ncols, int64_t *offsets_host)
{
    clear_error();
    SITING_REQUIRE(n >= 0, "siting_viewshed_layout: n < 0");
    SITING_REQUIRE(nrows >= 1 && ncols >= 1, "siting_viewshed_layout: empty terrain");
    SITING_REQUIRE(offsets_host != nullptr, "siting_viewshed_layout: offsets_host is NULL");
    SITING_REQUIRE(n == 0 || obs_host != nullptr, "siting_viewshed_layout: obs_host is NULL");
    int rc = validate_observers_host(obs_host, n, nrows, ncols, "siting_viewshed_layout");
    if (rc != SITING_OK)
        return rc;
    int64_t off = 0;
    for (int64_t i = 0; i < n; i++) {
        const siting_observer &o = obs_host[i];
        int64_t ylo = std::max<int64_t>(0, o.y - o.roi), yhi = std::min<int64_t>(nrows - 1, o.y + o.roi);
        int64_t xlo = std::max<int64_t>(0, o.x - o.roi), xhi = std::min<int64_t>(ncols - 1, o.x + o.roi);
        offsets_host[i] = off;
        off += (yhi - ylo + 1) * ((xhi >> 6) - (xlo >> 6) + 1);
    }
    offsets_host[n] = off;
    return off;
}

extern "C" int siting_viewshed_order(const siting_observer *obs_host, int64_t n,
                                     int32_t *order_host)
{
    clear_error();
    SITING_REQUIRE(n >= 0 && n <= INT32_MAX, "siting_viewshed_order: n out of range");
    SITING_REQUIRE(n == 0 || (obs_host && order_host), "siting_viewshed_order: NULL pointer");
    std::vector<int32_t> idx((size_t)n);
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](int32_t a, int32_t b) {
        return obs_host[a].roi > obs_host[b].roi;
    });
    std::copy(idx.begin(), idx.end(), order_host);
    return SITING_OK;
}
