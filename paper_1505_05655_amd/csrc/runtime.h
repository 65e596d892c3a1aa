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

// Largest VEC (1, 2, 4, or 8 when cap >= 8) the image pointers and the
// detector count allow. The plain correction kernels take up to 8 pixels per
// lane, the persistent batch kernel up to 4.
int max_vec(const uint16_t* dn, const uint16_t* out, int32_t detectors, int cap = 4);

// Launch shape with power-of-two strips of W detectors and about two rounds
// of resident tiles (the persistent batch and serving kernels tile requests
// this way; the plain path uses it for the L2 path).
void pow2_plan(int64_t lines, int32_t detectors, int32_t bands, int32_t levels, int vmax,
               const DeviceInfo& di, rc_plan* plan);

// Strips per band, strip bound W (power of two) and line chunk for about
// `target` equal tiles: strips of at least 64 detectors (or as many as fit
// `wmax`, the widest strip the LDS tile allows), whole units of `vec`
// detectors, then line chunks to reach the target. False if no tiling fits.
bool balanced_tiling(int64_t lines, int32_t detectors, int32_t bands, int vec, int wmax,
                     int64_t target, int32_t threads, int32_t unroll, int32_t* strips,
                     int32_t* strip, int32_t* chunk_lines);

// Widest power-of-two strip (<= 1024 detectors) whose LDS tile fits `budget`.
int widest_strip(int path, int levels, size_t budget);

// Levels for which rc_correct_ws encodes the LUT into its workspace, the
// workspace bytes that takes, and the plan it runs with.
bool ws_path(int32_t levels);
size_t dense_ws_bytes(int32_t detectors, int32_t bands, int32_t levels);
void ws_plan(int64_t lines, int32_t detectors, int32_t bands, int32_t levels, int vmax,
             const DeviceInfo& di, rc_plan* plan);

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

// Batch entries of the plan cache: the persistent batch kernel's tile shape
// (path, strip, vec of *plan) for requests of a class (levels,
// ceil(log2 detectors), largest usable vector width), as rc_batch_tune
// stores it.
bool tuned_batch_shape(int32_t detectors, int32_t levels, int vmax, const DeviceInfo& di,
                       rc_plan* plan);
void store_batch_shape(int32_t detectors, int32_t levels, int vmax, const DeviceInfo& di,
                       const rc_plan& plan, double us);

// Validation helpers.
bool overlaps(const void* a, size_t na, const void* b, size_t nb);
bool mul_ok(int64_t a, int64_t b, int64_t* r);

}  // namespace rc
