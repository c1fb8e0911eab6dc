// gn_step_static: the one-step entry point with its work buffer in a static
// device array, so that it allocates nothing.
//
// gn_step turns the caller's x into the library's state words in a buffer of
// the graph's workspace, which the first call on a graph allocates.  This
// variant keeps those words in `scratch`, a file-scope device array of
// kStaticMaxN words that every GPU the library runs on holds until the process
// ends.  Its device address is taken once per device (hipGetSymbolAddress,
// with that device current) and kept; the kernels receive that address, never
// the array's name, which in host code is only a host-side stand-in.
//
// Every call on one GPU shares that GPU's array: calls that overlap in time on
// one GPU (two streams, two threads) race on it.  Nothing in it needs clearing
// between calls: the conversion kernel writes all n words a call reads before
// the step kernel reads them, in stream order.
#include <mutex>

#include "gn_internal.h"

namespace {

constexpr int32_t kStaticMaxN = 1 << 21;   // 2,097,152 vertices: 8 MiB of state words
constexpr int kMaxDevices = 64;

__device__ __align__(256) float scratch[kStaticMaxN];

std::mutex g_scratch_mu;
float* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device `dev` (current), looked up on the first
// call for that device.
gn_status scratch_on(int dev, float** out) {
    if (dev < 0 || dev >= kMaxDevices) return GN_E_ARG;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return GN_E_HIP;
        }
        g_scratch_ptr[dev] = static_cast<float*>(p);
    }
    *out = g_scratch_ptr[dev];
    return GN_OK;
}

}  // namespace

extern "C" int32_t gn_step_static_max_n(void) { return kStaticMaxN; }

extern "C" gn_status gn_step_static(const gn_graph* g, float gamma, const float* x_in, float* x_out,
                                    hipStream_t stream) {
    gn_status st = gn_internal_step_args_ok(g, gamma, x_in, x_out);
    if (st != GN_OK || g->n == 0) return st;
    if (g->n > kStaticMaxN) return GN_E_SIZE;
    int dev = -1;
    GN_HIP_TRY(hipGetDevice(&dev));
    if (dev != g->device) return GN_E_ARG;   // the graph's arrays live on its own device
    float* y = nullptr;
    if ((st = scratch_on(dev, &y)) != GN_OK) return st;
    return gn_internal_step_with(g, gamma, x_in, x_out, y, stream);
}
