// Least-squares calibration fit (§III.B, case study 2 of the paper): per band
// b and detector d, the polynomial of order M that minimises the squared error
// over the points (x[b][i][d], y[b][i]), i < n, by the normal equations
// A a = B with A[j][k] = sum_i x_i^(j+k) (A[0][0] = n) and
// B[j] = sum_i x_i^j y_i, solved as a = A^-1 B, A^-1 from Gauss-Jordan
// elimination of [A | I] with partial pivoting (first row of largest
// magnitude). Binary64 throughout, no contraction: powers by repeated
// multiplication, sums in point order, so each detector's result is one fixed
// sequence of IEEE operations.
//
// One thread per (band, detector): a detector's n samples are read with loads
// that are coalesced across the wave (consecutive detectors), the band's
// targets are wave-uniform, and the (M+1) x (2M+2) system stays in registers
// (every index below is a compile-time constant after unrolling; the pivot
// row swap is a select, not an indexed access).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"
#include "rc.h"
#include "runtime.h"

namespace rc {

template <int M>
__device__ __forceinline__ void fit_one(const double* __restrict__ x,
                                        const double* __restrict__ y, int b, int d,
                                        int32_t points, int32_t detectors,
                                        double* __restrict__ coeffs) {
    constexpr int W = 2 * (M + 1);
    double S[2 * M + 1], T[M + 1];
#pragma unroll
    for (int k = 0; k <= 2 * M; ++k) S[k] = 0.0;
#pragma unroll
    for (int k = 0; k <= M; ++k) T[k] = 0.0;
    const double* xb = x + (size_t)b * (size_t)points * (size_t)detectors + (size_t)d;
    const double* yb = y + (size_t)b * (size_t)points;
    for (int i = 0; i < points; ++i) {
        const double xi = xb[(size_t)i * (size_t)detectors];
        const double yi = yb[i];
        double p = 1.0;  // x_i^k
#pragma unroll
        for (int k = 0; k <= 2 * M; ++k) {
            S[k] = S[k] + p;
            if (k <= M) T[k] = T[k] + p * yi;
            p = p * xi;
        }
    }
    double Mx[M + 1][W];
#pragma unroll
    for (int j = 0; j <= M; ++j) {
#pragma unroll
        for (int k = 0; k <= M; ++k) {
            Mx[j][k] = S[j + k];
            Mx[j][M + 1 + k] = j == k ? 1.0 : 0.0;
        }
    }
    bool singular = false;
#pragma unroll
    for (int c = 0; c <= M; ++c) {
        if (!singular) {
            int pr = c;
            double best = __builtin_fabs(Mx[c][c]);
#pragma unroll
            for (int r = c + 1; r <= M; ++r) {
                if (__builtin_fabs(Mx[r][c]) > best) {
                    best = __builtin_fabs(Mx[r][c]);
                    pr = r;
                }
            }
            if (!(best > 0.0)) {
                singular = true;
            } else {
#pragma unroll
                for (int r = c + 1; r <= M; ++r) {
                    if (r == pr) {
#pragma unroll
                        for (int k = 0; k < W; ++k) {
                            const double t = Mx[c][k];
                            Mx[c][k] = Mx[r][k];
                            Mx[r][k] = t;
                        }
                    }
                }
                const double piv = Mx[c][c];
#pragma unroll
                for (int k = 0; k < W; ++k) Mx[c][k] = Mx[c][k] / piv;
#pragma unroll
                for (int r = 0; r <= M; ++r) {
                    if (r == c) continue;
                    const double f = Mx[r][c];
#pragma unroll
                    for (int k = 0; k < W; ++k) Mx[r][k] = Mx[r][k] - f * Mx[c][k];
                }
            }
        }
    }
    double* a = coeffs + ((size_t)b * (size_t)detectors + (size_t)d) * 4;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        double v;
        if (singular) {
            v = __builtin_nan("");
        } else if (j > M) {
            v = 0.0;
        } else {
            v = 0.0;
#pragma unroll
            for (int k = 0; k <= M; ++k) v = v + Mx[j][M + 1 + k] * T[k];
        }
        a[j] = v;
    }
}

template <int M>
__global__ __launch_bounds__(256) void k_fit(const double* __restrict__ x,
                                             const double* __restrict__ y, int32_t bands,
                                             int32_t points, int32_t detectors,
                                             double* __restrict__ coeffs) {
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= detectors) return;
    for (int b = blockIdx.y; b < bands; b += gridDim.y)
        fit_one<M>(x, y, b, d, points, detectors, coeffs);
}

hipError_t launch_fit(const double* x, const double* y, int32_t bands, int32_t points,
                      int32_t detectors, int32_t order, double* coeffs, hipStream_t stream) {
    const dim3 grid((unsigned)((detectors + 255) / 256),
                    (unsigned)(bands < 65535 ? bands : 65535));  // grid-stride over bands beyond
    auto k = order == 0 ? k_fit<0> : order == 1 ? k_fit<1> : order == 2 ? k_fit<2> : k_fit<3>;
    hipLaunchKernelGGL(k, grid, dim3(256), 0, stream, x, y, bands, points, detectors, coeffs);
    return hipGetLastError();
}

}  // namespace rc

using namespace rc;

extern "C" {

rc_status rc_fit(const double* x, const double* y, int32_t bands, int32_t points,
                 int32_t detectors, int32_t order, double* coeffs, hipStream_t stream) {
    if (bands < 0 || detectors < 0 || order < 0 || order > 3 || points < order + 1)
        return RC_EINVAL;
    int64_t rows = 0, xn = 0, yn = 0;
    if (!mul_ok(bands, detectors, &rows) || !mul_ok(rows, points, &xn) ||
        !mul_ok(bands, points, &yn) || xn > INT64_MAX / 8 || rows > INT64_MAX / 32)
        return RC_EINVAL;
    if (rows == 0) return RC_OK;
    if (!x || !y || !coeffs) return RC_EINVAL;
    if (((uintptr_t)x | (uintptr_t)y | (uintptr_t)coeffs) & 7u) return RC_EINVAL;
    if (overlaps(coeffs, (size_t)rows * 32, x, (size_t)xn * 8) ||
        overlaps(coeffs, (size_t)rows * 32, y, (size_t)yn * 8))
        return RC_EINVAL;
    if (!current_device()) return RC_EHIP;
    hipError_t e = launch_fit(x, y, bands, points, detectors, order, coeffs, stream);
    return e == hipSuccess ? RC_OK : hip_fail(e);
}

}  // extern "C"
