// Reference CPU implementation of look-up-table generation and image correction.
//
// TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the
// benchmark's CPU-baseline leg, never by the GPU library. Plain, single
// threaded, slow on purpose: every loop follows the definition in oracle.hpp
// with no blocking, fusion or reordering.
//
// Built with the host compiler and -O2 -ffp-contract=off -fno-fast-math on
// x86-64 (SSE2 binary64, so every + and * below is one correctly rounded
// IEEE-754 operation and nothing is fused into an FMA).
//
// Paper: Banerjee & Dave, "GPGPU Based Parallelized Client-Server Framework
// for Providing High Performance Computation Support", §I, which names LUT
// generation and image correction as the task; the paper gives no formula,
// so the definition in oracle.hpp is the one this project fixes.
#include "oracle.hpp"

#include <cmath>
#include <cstddef>

extern "C" {

uint16_t oracle_lut_entry(const double* a, int32_t v, int32_t levels) {
    // The level is an integer below 2^16, so the conversion is exact.
    const double x = (double)v;
    // Horner from the cubic coefficient down; one rounding per operation.
    double acc = a[3];
    acc = acc * x;
    acc = acc + a[2];
    acc = acc * x;
    acc = acc + a[1];
    acc = acc * x;
    acc = acc + a[0];
    // C round(): nearest integer, halfway cases away from zero. Exact.
    const double r = std::round(acc);
    // Clamp in binary64 before converting; NaN fails the first test.
    if (!(r > 0.0)) return 0;
    const double top = (double)(levels - 1);
    if (r >= top) return (uint16_t)(levels - 1);
    return (uint16_t)r;
}

void oracle_lut_build(const double* coeffs, int32_t bands, int32_t detectors,
                      int32_t levels, uint16_t* lut) {
    for (int32_t b = 0; b < bands; ++b) {
        for (int32_t d = 0; d < detectors; ++d) {
            const size_t row = (size_t)b * (size_t)detectors + (size_t)d;
            const double* a = coeffs + row * 4;
            for (int32_t v = 0; v < levels; ++v) {
                lut[row * (size_t)levels + (size_t)v] = oracle_lut_entry(a, v, levels);
            }
        }
    }
}

void oracle_correct(const uint16_t* dn, const uint16_t* lut, int64_t lines,
                    int32_t detectors, int32_t bands, int32_t levels,
                    uint16_t* out) {
    const uint16_t top = (uint16_t)(levels - 1);
    for (int32_t b = 0; b < bands; ++b) {
        for (int64_t n = 0; n < lines; ++n) {
            for (int32_t d = 0; d < detectors; ++d) {
                const size_t pix = ((size_t)b * (size_t)lines + (size_t)n) * (size_t)detectors
                                   + (size_t)d;
                uint16_t v = dn[pix];
                if (v > top) v = top;
                const size_t row = (size_t)b * (size_t)detectors + (size_t)d;
                out[pix] = lut[row * (size_t)levels + (size_t)v];
            }
        }
    }
}

void oracle_pixel(const double* coeffs, const uint16_t* dn, int64_t lines,
                  int32_t detectors, int32_t bands, int32_t levels,
                  uint16_t* out) {
    for (int32_t b = 0; b < bands; ++b) {
        for (int64_t n = 0; n < lines; ++n) {
            for (int32_t d = 0; d < detectors; ++d) {
                const size_t pix = ((size_t)b * (size_t)lines + (size_t)n) * (size_t)detectors
                                   + (size_t)d;
                int32_t v = dn[pix];
                if (v > levels - 1) v = levels - 1;
                const double* a = coeffs + ((size_t)b * (size_t)detectors + (size_t)d) * 4;
                out[pix] = oracle_lut_entry(a, v, levels);
            }
        }
    }
}

}  // extern "C"
