// Linear device-to-device copy with the access widths and cache policies of
// the correction kernels: the practical streaming ceiling the correction is
// measured against (2 B read + 2 B written per pixel and no LUT is what a
// copy of the image moves).
//
// Each workgroup iteration moves one contiguous block of threads x unroll x
// 16 bytes: lane t of the block loads 16 bytes at (u * threads + t) * 16 for
// u < unroll (every wave instruction covers 1 KiB), all unroll loads are in
// flight before the first store, and the workgroups of a persistent grid
// (wgs_per_cu per CU) stride over the blocks. The tail (less than one block)
// is copied by the same loop with per-lane guards.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "rc.h"
#include "runtime.h"

namespace rc {

namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <int POLICY>
__device__ __forceinline__ u32x4 ld16(const u32x4* p) {
    if constexpr (POLICY == 1) return __builtin_nontemporal_load(p);
    else return *p;
}

template <int POLICY>
__device__ __forceinline__ void st16(u32x4* p, u32x4 v) {
    if constexpr (POLICY == 1 || POLICY == 2) __builtin_nontemporal_store(v, p);
    else *p = v;
}

template <int UNROLL, int POLICY>
__global__ __launch_bounds__(1024) void k_stream_copy(const u32x4* __restrict__ src,
                                                      u32x4* __restrict__ dst, size_t n16) {
    const size_t nt = blockDim.x;
    const size_t block = nt * UNROLL;
    const size_t full = n16 / block;
    for (size_t blk = blockIdx.x; blk < full; blk += gridDim.x) {
        const size_t base = blk * block + threadIdx.x;
        u32x4 v[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) v[u] = ld16<POLICY>(src + base + u * nt);
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) st16<POLICY>(dst + base + u * nt, v[u]);
    }
    // The last partial block: the workgroup that would have taken it next.
    if (blockIdx.x == full % gridDim.x) {
        for (size_t i = full * block + threadIdx.x; i < n16; i += nt) st16<POLICY>(dst + i, ld16<POLICY>(src + i));
    }
}

__global__ void k_copy_bytes(const unsigned char* __restrict__ src, unsigned char* __restrict__ dst,
                             size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

typedef void (*CopyKernel)(const u32x4*, u32x4*, size_t);

CopyKernel pick(int unroll, int policy) {
    if (unroll == 4) {
        if (policy == 0) return k_stream_copy<4, 0>;
        if (policy == 1) return k_stream_copy<4, 1>;
        return k_stream_copy<4, 2>;
    }
    if (unroll == 8) {
        if (policy == 0) return k_stream_copy<8, 0>;
        if (policy == 1) return k_stream_copy<8, 1>;
        return k_stream_copy<8, 2>;
    }
    if (policy == 0) return k_stream_copy<2, 0>;
    if (policy == 1) return k_stream_copy<2, 1>;
    return k_stream_copy<2, 2>;
}

}  // namespace
}  // namespace rc

using namespace rc;

extern "C" rc_status rc_stream_copy(const void* src, void* dst, size_t bytes,
                                    const rc_copy_plan* plan, hipStream_t stream) {
    if (bytes == 0) return RC_OK;
    if (!src || !dst) return RC_EINVAL;
    if (((uintptr_t)src | (uintptr_t)dst) & 15u) return RC_EINVAL;
    if (overlaps(src, bytes, dst, bytes)) return RC_EINVAL;
    rc_copy_plan p;
    if (plan) {
        p = *plan;
    } else {
        p.threads = 256;
        p.unroll = 4;
        p.policy = 1;
        p.wgs_per_cu = 8;
    }
    if (p.threads != 256 && p.threads != 512 && p.threads != 1024) return RC_EINVAL;
    if (p.unroll != 2 && p.unroll != 4 && p.unroll != 8) return RC_EINVAL;
    if (p.policy < 0 || p.policy > 2) return RC_EINVAL;
    if (p.wgs_per_cu < 1 || p.wgs_per_cu * p.threads > 2048) return RC_EINVAL;
    const DeviceInfo* di = current_device();
    if (!di) return RC_EHIP;
    const size_t n16 = bytes / 16;
    if (n16 > 0) {
        const size_t blocks = (n16 + (size_t)p.threads * p.unroll - 1) / ((size_t)p.threads * p.unroll);
        const size_t grid = std::min<size_t>(blocks, (size_t)std::max(1, di->cus) * p.wgs_per_cu);
        hipLaunchKernelGGL(pick(p.unroll, p.policy), dim3((unsigned)grid), dim3(p.threads), 0, stream,
                           (const u32x4*)src, (u32x4*)dst, n16);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e);
    }
    const size_t tail = bytes - n16 * 16;
    if (tail) {
        hipLaunchKernelGGL(k_copy_bytes, dim3(1), dim3(16), 0, stream,
                           (const unsigned char*)src + n16 * 16, (unsigned char*)dst + n16 * 16, tail);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e);
    }
    return RC_OK;
}
