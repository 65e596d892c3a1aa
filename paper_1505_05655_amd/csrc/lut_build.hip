// LUT build kernel (LUT generation, a task named in §I): every entry of
// lut[b][d][v] from the binary64 calibration polynomial of (b, d).
//
// One thread computes 8 consecutive levels of one LUT row and writes them
// with a single 16-byte store when the row pitch allows it. For rows of 512
// levels or more, a wave evaluates whole rows, 512 consecutive levels per
// pass, so the row index and the row's coefficients are wave-uniform (scalar
// loads, no per-lane index arithmetic) and each wave store writes 1 KiB
// contiguously.
// The arithmetic is the fixed, uncontracted binary64 sequence of
// rc::lut_entry, so every entry is bit-identical to the CPU definition.
#include "device_ops.h"
#include "kernels.h"

namespace rc {

__global__ __launch_bounds__(256) void k_lut_build(const double* __restrict__ coeffs, int64_t rows,
                                                   int32_t levels, int32_t chunks,
                                                   int32_t log_chunks, int32_t vec,
                                                   uint16_t* __restrict__ lut) {
    const int64_t total = rows * (int64_t)chunks;
    const double lim = (double)levels;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        // Row and 8-level chunk of this thread (a shift when chunks is 2^k).
        const int64_t row = log_chunks >= 0 ? (t >> log_chunks) : t / chunks;
        const int c = (int)(t - row * chunks);
        const double* a = coeffs + row * 4;
        const double a0 = a[0], a1 = a[1], a2 = a[2], a3 = a[3];
        const int v0 = c * 8;
        uint16_t* dst = lut + row * (int64_t)levels + v0;
        if (vec) {
            uint32_t e[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) e[k] = lut_entry(a0, a1, a2, a3, v0 + k, lim);
            u32x4 q;
            q.x = e[0] | (e[1] << 16);
            q.y = e[2] | (e[3] << 16);
            q.z = e[4] | (e[5] << 16);
            q.w = e[6] | (e[7] << 16);
            *(u32x4*)dst = q;
        } else {
            for (int k = 0; k < 8 && v0 + k < levels; ++k) {
                dst[k] = (uint16_t)lut_entry(a0, a1, a2, a3, v0 + k, lim);
            }
        }
    }
}

// Wave w of the grid evaluates row w (then w + number of waves, ...), 512
// levels per pass. nt: non-temporal 16-byte stores, for LUTs larger than the
// L2 caches, which the correction after the build does not find there anyway
// (on the 3 x 50000 x 6000 scene the correction after a build took 0.77 ms
// instead of 0.83 ms on one GPU, and the same 0.82-0.84 ms either way on two
// others; the build itself is not slower).
__global__ __launch_bounds__(256) void k_lut_build_rows(const double* __restrict__ coeffs,
                                                        int64_t rows, int32_t levels, int32_t vec,
                                                        int32_t nt, uint16_t* __restrict__ lut) {
    const int lane = threadIdx.x & 63;
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
    const double lim = (double)levels;
    for (int64_t row = (int64_t)blockIdx.x * (blockDim.x >> 6) +
                       __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
         row < rows; row += nwaves) {
        const double* a = coeffs + row * 4;
        const double a0 = a[0], a1 = a[1], a2 = a[2], a3 = a[3];
        uint16_t* dst_row = lut + row * (int64_t)levels;
        for (int v0 = lane * 8; v0 < levels; v0 += 512) {
            const int n = min(8, levels - v0);
            uint16_t* dst = dst_row + v0;
            if (vec && n == 8) {
                uint32_t e[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) e[k] = lut_entry(a0, a1, a2, a3, v0 + k, lim);
                u32x4 q;
                q.x = e[0] | (e[1] << 16);
                q.y = e[2] | (e[3] << 16);
                q.z = e[4] | (e[5] << 16);
                q.w = e[6] | (e[7] << 16);
                if (nt) __builtin_nontemporal_store(q, (u32x4*)dst);
                else *(u32x4*)dst = q;
            } else {
                for (int k = 0; k < n; ++k) dst[k] = (uint16_t)lut_entry(a0, a1, a2, a3, v0 + k, lim);
            }
        }
    }
}

hipError_t launch_lut_build(const double* coeffs, int64_t rows, int32_t levels, uint16_t* lut,
                            hipStream_t stream) {
    const bool vec = (levels % 8 == 0) && (((uintptr_t)lut & 15u) == 0);
    if (levels >= 512) {
        int64_t blocks = (rows + 3) / 4;  // one wave per row
        if (blocks > (int64_t)1 << 20) blocks = (int64_t)1 << 20;  // grid-stride beyond this
        // Non-temporal above the GPU's aggregate L2 (8 XCDs x 4 MiB).
        const int nt = (double)rows * (double)levels * 2.0 > (double)(32u << 20) ? 1 : 0;
        hipLaunchKernelGGL(k_lut_build_rows, dim3((unsigned)blocks), dim3(256), 0, stream, coeffs,
                           rows, levels, vec ? 1 : 0, nt, lut);
        return hipGetLastError();
    }
    const int32_t chunks = (levels + 7) / 8;
    int32_t log_chunks = -1;
    if ((chunks & (chunks - 1)) == 0) {
        log_chunks = 0;
        while ((1 << log_chunks) < chunks) ++log_chunks;
    }
    const int64_t total = rows * (int64_t)chunks;
    const int threads = 256;
    int64_t blocks = (total + threads - 1) / threads;
    if (blocks > (int64_t)1 << 20) blocks = (int64_t)1 << 20;  // grid-stride beyond this
    hipLaunchKernelGGL(k_lut_build, dim3((unsigned)blocks), dim3(threads), 0, stream, coeffs, rows,
                       levels, chunks, log_chunks, vec ? 1 : 0, lut);
    return hipGetLastError();
}

}  // namespace rc
