// d4dgs_bin_sort_noalloc: the binning and per-tile sort of d4dgs_bin_sort with its
// workspace in a static device array of the library, for callers that cannot allocate
// device memory.  Every GPU the library runs on holds its own copy of the array until the
// process ends.  In host code the array's name stands for a host-side shadow, not a device
// address: its device address is looked up once per device (hipGetSymbolAddress, with that
// device current) and only that address is handed to kernels.
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "internal.hpp"

namespace d4 {

namespace {

static_assert(D4DGS_STATIC_SCRATCH_BYTES % 256 == 0, "the scratch is carved in 256-byte steps");

__device__ __align__(256) unsigned char scratch[D4DGS_STATIC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
std::vector<void *> g_scratch_ptr;  // device address of `scratch`, per device (NULL: not looked up)

// The current device's copy of `scratch`, looked up on the first call on that device.
hipError_t device_scratch(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace

}  // namespace d4

using namespace d4;

extern "C" d4dgs_status d4dgs_bin_sort_noalloc(const d4dgs_splats *splats, int32_t n, int32_t width, int32_t height,
                                               d4dgs_bins *bins, int32_t *d_status, d4dgs_stream stream) {
    if (n < 0) {
        set_error("bin_sort_noalloc: n < 0");
        return D4DGS_ERR_INVALID_ARG;
    }
    if (!bins || bins->capacity < 1 || bins->capacity > (int64_t)0x7fffffff) {
        set_error("bin_sort_noalloc: bins NULL or capacity outside [1, 2^31)");
        return D4DGS_ERR_INVALID_ARG;
    }
    size_t need = 0;
    const d4dgs_status s = d4dgs_workspace_size(n, width, height, bins->capacity, &need);
    if (s != D4DGS_OK) return s;
    if (need > (size_t)D4DGS_STATIC_SCRATCH_BYTES) {
        set_error("bin_sort_noalloc: n = " + std::to_string(n) + ", " + std::to_string(width) + "x" +
                  std::to_string(height) + " and capacity " + std::to_string(bins->capacity) + " need " +
                  std::to_string(need) + " bytes of scratch; the static scratch holds " +
                  std::to_string((size_t)D4DGS_STATIC_SCRATCH_BYTES));
        return D4DGS_ERR_OUT_OF_MEMORY;
    }
    void *ws = nullptr;
    const hipError_t e = device_scratch(&ws);
    if (e != hipSuccess) {
        set_error(std::string("bin_sort_noalloc: static scratch: ") + hipGetErrorString(e));
        return D4DGS_ERR_HIP;
    }
    // d4dgs_bin_sort clears the tile counters in its first kernel, so the array's contents
    // from an earlier call need no clearing here
    return d4dgs_bin_sort(splats, n, width, height, ws, (size_t)D4DGS_STATIC_SCRATCH_BYTES, bins, d_status, stream);
}
