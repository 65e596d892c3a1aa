// rc_correct_noalloc: rc_correct_ws with the library's own scratch instead
// of a caller workspace, for callers that cannot allocate device memory.
//
// The scratch is one file-scope device array per GPU the library runs on
// (held until the process ends). Host code never passes the array's name to
// a kernel: its device address is read once per device with
// hipGetSymbolAddress (with that device current) and kept; kernels receive
// that address. Every call on a GPU shares that GPU's array, so calls that
// overlap on one GPU race; the array keeps the last call's contents, and
// nothing in it needs to start at zero (the encode kernel writes every block
// the correction then reads).
#include <hip/hip_runtime.h>

#include <mutex>

#include "rc.h"
#include "runtime.h"

namespace rc {

namespace {

static __device__ __align__(256) unsigned char scratch[RC_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
void* g_ptr[kMaxDevices];
std::mutex g_mu;

// The device address of this GPU's scratch; NULL (and the HIP error kept)
// if it cannot be read.
void* scratch_ptr(int dev) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol);
            return nullptr;
        }
        g_ptr[dev] = p;
    }
    return g_ptr[dev];
}

}  // namespace
}  // namespace rc

using namespace rc;

extern "C" rc_status rc_correct_noalloc(const uint16_t* dn, const uint16_t* lut, int64_t lines,
                                        int32_t detectors, int32_t bands, int32_t levels,
                                        uint16_t* out, hipStream_t stream) {
    const size_t need = rc_correct_ws_bytes(detectors, bands, levels);
    if (need == 0)  // no workspace for this shape: the plain call
        return rc_correct(dn, lut, lines, detectors, bands, levels, out, stream);
    if (need > (size_t)RC_NOALLOC_SCRATCH_BYTES) return RC_EINVAL;
    int dev = 0;
    if (!current_device(&dev)) return RC_EHIP;
    void* ws = scratch_ptr(dev);
    if (!ws) return RC_EHIP;
    return rc_correct_ws(dn, lut, lines, detectors, bands, levels, out, ws,
                         (size_t)RC_NOALLOC_SCRATCH_BYTES, nullptr, stream);
}
