// Host-visible launch interface of the HIP kernels (internal to librc).
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include "rc.h"

namespace rc {

// Longest LUT rows the dense LDS strip encodes (16-bit block headers).
constexpr int kDenseMaxLevels = 8192;
// Most threads per workgroup of the dense path (its kernels' launch bound).
constexpr int kDenseMaxThreads = 512;

// Everything the correction kernel needs to decode a tile id.
struct ApplyParams {
    const uint16_t* dn;
    const uint16_t* lut;
    uint16_t* out;
    int64_t lines;       // N
    int32_t detectors;   // D
    int32_t levels;      // L
    int32_t bands;       // B
    int32_t log_strip;   // log2(W): LDS tile width, widest strip
    int32_t strips;      // strips per band: ceil(D / W), or the plan's count when uneven
    int32_t uneven;      // 1: strip s is detector units [s*U/strips, (s+1)*U/strips) with
                         //    U = D / vec (units of vec detectors); 0: strip s is [s*W, s*W+W)
    int32_t vec;         // pixels per lane (the unit of uneven strips)
    int32_t dense;       // lanes per strip line: 0 W / vec, 1 strip width / vec
    int32_t chunks;      // ceil(N / chunk_lines)
    int64_t chunk_lines;
    int32_t ntiles;      // bands * strips * chunks
    int32_t xcds;        // 0/1: identity tile order, else the XCD count
    int32_t chunk_major; // 0: strips vary fastest, 1: line chunks vary fastest
    int32_t interleave;  // 1: line chunk c of `chunks` is every chunks-th pass from pass c
    int32_t lut_vec;     // LUT rows may be staged with 16-byte loads
    // Dense tiles: the strip's blocks already encoded by k_dense_encode
    // (layout [bands][blocks][detectors]); NULL: each tile encodes its strip.
    const uint64_t* pre_planes;
    const int16_t* pre_heads;
    int32_t threads;     // threads that stream the image (the plan's workgroup size)
    int32_t block;       // threads launched: `threads`, or more whose waves only stage
};

// Encodes every 64-level block of every LUT row into the dense form (planes
// and headers, [bands][ceil(levels / 64)][detectors]; a block that does not
// fit the form gets the header kDenseBad).
hipError_t launch_dense_encode(const uint16_t* lut, int32_t bands, int32_t detectors,
                               int32_t levels, uint64_t* planes, int16_t* heads,
                               hipStream_t stream);

// LUT build that also writes each row's dense encoding ([bands][blocks]
// [detectors] planes and heads, as launch_dense_encode): one wave per row.
hipError_t launch_lut_build_ws(const double* coeffs, int64_t rows, int32_t detectors,
                               int32_t levels, uint16_t* lut, uint64_t* planes, int16_t* heads,
                               hipStream_t stream);

// lut_build: one thread per 8 consecutive levels of one LUT row.
hipError_t launch_lut_build(const double* coeffs, int64_t rows, int32_t levels, uint16_t* lut,
                            hipStream_t stream);

// Least-squares calibration fit of order 0..3 (arguments validated by rc_fit).
hipError_t launch_fit(const double* x, const double* y, int32_t bands, int32_t points,
                      int32_t detectors, int32_t order, double* coeffs, hipStream_t stream);

// Bilinear Bayer demosaicing (arguments validated by rc_demosaic).
hipError_t launch_demosaic(const uint16_t* raw, int32_t images, int32_t H, int32_t W,
                           uint16_t* rgb, int cus, hipStream_t stream);

// Gradient-based (adaptive colour plane) demosaicing (arguments validated by
// rc_demosaic_gradient).
hipError_t launch_demosaic_gradient(const uint16_t* raw, int32_t images, int32_t H, int32_t W,
                                    uint16_t* rgb, int cus, hipStream_t stream);

// Correction with the given plan (already validated).
hipError_t launch_apply(const ApplyParams& p, const rc_plan& plan, size_t lds_bytes,
                        hipStream_t stream);

// Raise the dynamic-LDS limit of every correction kernel on the current
// device (once per device) as far as `bytes` of LDS per workgroup allows;
// `usable` receives the dynamic LDS every kernel can then launch with.
hipError_t prepare_apply_kernels(size_t bytes, size_t* usable);

}  // namespace rc
