// Host runtime shared by the C-ABI entry points (internal to librc).
#pragma once

#include <hip/hip_runtime_api.h>
#include <stddef.h>
#include <stdint.h>

#include <string>

#include "kernels.h"
#include "rc.h"

namespace rc {

// Static properties of one device, read once.
struct DeviceInfo {
    int cus = 0;          // compute units
    int xcds = 1;         // accelerator complex dies (separate L2s)
    size_t lds = 0;       // max dynamic LDS per workgroup, bytes
    size_t lds_per_cu = 0;
    std::string arch;     // e.g. "gfx950"
    size_t hbm_bytes = 0;
};

// Info for the current device; NULL (and last HIP error set) on failure.
const DeviceInfo* current_device(int* dev_out = nullptr);

// Records `e` as this thread's last HIP error and returns RC_EHIP.
rc_status hip_fail(hipError_t e);

// Largest VEC the image pointers and the detector count allow (1, 2 or 4).
int max_vec(const uint16_t* dn, const uint16_t* out, int32_t detectors);

// Default launch shape for a shape class (no tuning).
void default_plan(int64_t lines, int32_t detectors, int32_t bands, int32_t levels, int vmax,
                  const DeviceInfo& di, rc_plan* plan);

// Checks a plan against a shape and device; fills `p` and `lds_bytes`.
rc_status check_plan(const rc_plan& plan, int64_t lines, int32_t detectors, int32_t bands,
                     int32_t levels, int vmax, const DeviceInfo& di, ApplyParams* p,
                     size_t* lds_bytes);

// Longest line chunk a tile may have (32-bit buffer offsets); < 1 if none fits.
int64_t max_chunk_lines(int32_t detectors, int32_t threads, int32_t unroll);

// LDS bytes a plan's tile needs (0 for the L2 path).
size_t plan_lds_bytes(int path, int strip, int levels);

// Concurrent workgroups of one plan on the whole device.
int plan_slots(const rc_plan& plan, size_t lds_bytes, const DeviceInfo& di);

// Tuned plan from the plan cache, if one matches the shape class.
bool tuned_plan(int64_t lines, int32_t detectors, int32_t bands, int32_t levels, int vmax,
                const DeviceInfo& di, rc_plan* plan);

// Validation helpers.
bool overlaps(const void* a, size_t na, const void* b, size_t nb);
bool mul_ok(int64_t a, int64_t b, int64_t* r);

}  // namespace rc
