// The segmented map-reduce for callers that cannot allocate device memory
// (code under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc): its tile table and tile partials live in a static device array
// of this library instead of a caller-owned workspace.
//
// The array is a device symbol of this translation unit.  Its host-side name
// is only a stand-in for the symbol, so host code never passes it to a
// kernel: the device address is taken once per device with
// hipGetSymbolAddress, with that device current, and only that address is
// used afterwards.  Each device holds its own copy until the process ends.
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.h"

namespace {

constexpr size_t kScratchBytes = HIPMR_NOALLOC_SCRATCH_BYTES;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once per
// device).
hipmr_status scratch_on_current_device(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return hipmr::fail(HIPMR_E_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return hipmr::fail(HIPMR_E_HIP, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return hipmr::fail(HIPMR_E_HIP, std::string("hipGetSymbolAddress(scratch): ") +
                                                hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return HIPMR_OK;
}

struct NoAllocScope {
    NoAllocScope() { hipmr::set_no_alloc(true); }
    ~NoAllocScope() { hipmr::set_no_alloc(false); }
};

}  // namespace

extern "C" {

size_t hipmr_noalloc_scratch_bytes(void) { return kScratchBytes; }

hipmr_status hipmr_reduce_segmented_noalloc(hipmr_handle h, const char* combine, const char* neutral,
                                            int32_t nseg, const int64_t* d_offsets, int64_t total_n,
                                            void* const* args, void* d_out,
                                            const hipmr_launch_config* cfg, void* stream) {
    hipmr::clear_error();
    if (!h) return hipmr::fail(HIPMR_E_INVALID, "NULL handle");
    if (nseg < 0 || total_n < 0) return hipmr::fail(HIPMR_E_INVALID, "nseg and total_n must be >= 0");
    const size_t need = hipmr::segmented_workspace(h, nseg, total_n);
    if (need > kScratchBytes)
        return hipmr::fail(HIPMR_E_WORKSPACE,
                           "hipmr_reduce_segmented_noalloc: " + std::to_string(nseg) + " segments over " +
                               std::to_string(total_n) + " elements need " + std::to_string(need) +
                               " bytes of scratch, more than the " + std::to_string(kScratchBytes) +
                               " bytes of the static scratch array; use hipmr_reduce_segmented "
                               "with a workspace");
    void* ws = nullptr;
    if (nseg > 0) {
        hipmr_status st = scratch_on_current_device(&ws);
        if (st != HIPMR_OK) return st;
    }
    NoAllocScope scope;
    return hipmr::reduce_segmented_on(h, combine, neutral, nseg, d_offsets, total_n, args, d_out, ws,
                                      kScratchBytes, cfg, stream);
}

}  // extern "C"
