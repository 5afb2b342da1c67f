// ForceAtlas2 layout for callers that cannot allocate device memory (code under HIP
// graph capture, tight serving loops, hosts that forbid hipMalloc): the same kernels
// and results as bgv_fa2_layout, with the scratch taken from a fixed device array of
// this library instead of a caller workspace.
//
// The array is a file-scope __device__ object: every GPU the library runs on holds its
// own copy, at its own address, until the process ends.  Host code may not use the
// array's name as a device address (it names a host-side stand-in), so the address is
// looked up once per device with hipGetSymbolAddress and kept here; kernels receive
// that address as their workspace pointer.
#include <mutex>

#include "common.h"
#include "fa2_internal.h"

namespace bgv {
namespace {

__device__ __align__(256) char scratch[BGV_FA2_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
void *g_scratch_addr[kMaxDevices];
std::mutex g_scratch_mu;

// Device address of the current device's copy of `scratch`, looked up on first use.
bgv_status scratch_address(void **out) {
    int dev = -1;
    BGV_CHECK_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("bgv_fa2_layout_static: device %d is beyond the %d devices this library tracks", dev,
                  kMaxDevices);
        return BGV_E_INVALID;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_addr[dev] == nullptr) {
        void *p = nullptr;
        BGV_CHECK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (p == nullptr || (reinterpret_cast<uintptr_t>(p) & 255u) != 0) {
            set_error("bgv_fa2_layout_static: scratch array of device %d at %p is not usable", dev, p);
            return BGV_E_HIP;
        }
        g_scratch_addr[dev] = p;
    }
    *out = g_scratch_addr[dev];
    return BGV_OK;
}

}  // namespace
}  // namespace bgv

using namespace bgv;

extern "C" bgv_status bgv_fa2_layout_static(int32_t K, int64_t E, const int32_t *edges, const float *attr_w,
                                            const float *mass, float *pos, float *fprev, float *speed,
                                            const bgv_fa2_params *p, bgv_stream_t stream) {
    clear_error();
    const size_t need = bgv_fa2_workspace(K, E, p);
    if (need == 0) {
        set_error("bgv_fa2_layout_static: invalid arguments (K=%d E=%lld)", K, (long long)E);
        return BGV_E_INVALID;
    }
    if (need > (size_t)BGV_FA2_STATIC_SCRATCH_BYTES) {
        set_error("bgv_fa2_layout_static: K=%d, E=%lld needs %zu bytes of scratch, more than the %zu this entry "
                  "point holds; use bgv_fa2_layout with a caller workspace",
                  K, (long long)E, need, (size_t)BGV_FA2_STATIC_SCRATCH_BYTES);
        return BGV_E_INVALID;
    }
    if ((E > 0 && !edges) || !pos || !fprev || !speed) {
        set_error("bgv_fa2_layout_static: null pointer");
        return BGV_E_INVALID;
    }
    void *ws = nullptr;
    BGV_TRY(scratch_address(&ws));
    // on the caller's stream alone: no second stream or events are created
    return fa2_layout_run(K, E, edges, attr_w, mass, pos, fprev, speed, p, ws, (size_t)BGV_FA2_STATIC_SCRATCH_BYTES,
                          stream, false);
}
