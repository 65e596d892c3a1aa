// Device-side building blocks of the LUT build and correction kernels:
// the binary64 LUT entry, the XCD-aware tile order and the two tile bodies
// (LDS-staged strip and L2-resident global gather). Shared by the plain
// kernels (lut_build.hip, lut_apply.hip) and the persistent batch kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

// The LUT entry is a fixed sequence of binary64 operations: no contraction
// into fused multiply-adds anywhere in this translation unit (the build also
// passes -ffp-contract=off).
#pragma clang fp contract(off)

namespace rc {

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// LUT entry for integer level v (§I LUT generation, definition in rc.h):
// Horner from the cubic coefficient down, then C round() (halfway away from
// zero, exact), then the clamp to [0, top] done in binary64 before converting.
__device__ __forceinline__ uint32_t lut_entry(double a0, double a1, double a2, double a3, int v,
                                              double top) {
    const double x = (double)v;
    double acc = a3;
    acc = acc * x;
    acc = acc + a2;
    acc = acc * x;
    acc = acc + a1;
    acc = acc * x;
    acc = acc + a0;
    const double r = __builtin_round(acc);
    if (!(r > 0.0)) return 0u;  // negatives, -0, NaN
    if (r >= top) return (uint32_t)top;
    return (uint32_t)r;
}

// Workgroups are dispatched round-robin over the XCDs (block i runs on XCD
// i mod X). Renumber them so that XCD x receives one contiguous range of
// logical tiles: neighbouring tiles then share that XCD's L2.
__device__ __forceinline__ int xcd_tile(int i, int G, int X) {
    if (X <= 1) return i;
    const int q = G / X, r = G - (G / X) * X;
    const int x = i % X, k = i / X;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + k;
}

template <typename T, bool NTH>
__device__ __forceinline__ T load_px(const T* p) {
    if constexpr (NTH) return __builtin_nontemporal_load(p);
    else return *p;
}

template <typename T, bool NTH>
__device__ __forceinline__ void store_px(T* p, T v) {
    if constexpr (NTH) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// VEC pixels of one line held by one lane.
template <int VEC> struct Px;
template <> struct Px<1> { typedef unsigned short T; };
template <> struct Px<2> { typedef unsigned int T; };
template <> struct Px<4> { typedef u32x2 T; };

// Gather of one 16-bit DN through an LDS strip tile laid out level-major:
// tile[v * W + j] is detector j's entry for level v.
__device__ __forceinline__ uint32_t g_lds(const uint16_t* tile, uint32_t dnv, uint32_t top,
                                          int logW, int j) {
    const uint32_t v = dnv < top ? dnv : top;
    return tile[(v << logW) + j];
}

// Gather from a global LUT row.
__device__ __forceinline__ uint32_t g_glb(const uint16_t* row, uint32_t dnv, uint32_t top) {
    const uint32_t v = dnv < top ? dnv : top;
    return row[v];
}

template <int VEC> struct Gather;

template <> struct Gather<1> {
    __device__ static __forceinline__ unsigned short lds(unsigned short w, const uint16_t* t,
                                                         uint32_t top, int logW, int j) {
        return (unsigned short)g_lds(t, w, top, logW, j);
    }
    __device__ static __forceinline__ unsigned short glb(unsigned short w, const uint16_t* row,
                                                         size_t L, uint32_t top) {
        (void)L;
        return (unsigned short)g_glb(row, w, top);
    }
};

template <> struct Gather<2> {
    __device__ static __forceinline__ unsigned int lds(unsigned int w, const uint16_t* t,
                                                       uint32_t top, int logW, int j) {
        return g_lds(t, w & 0xffffu, top, logW, j) | (g_lds(t, w >> 16, top, logW, j + 1) << 16);
    }
    __device__ static __forceinline__ unsigned int glb(unsigned int w, const uint16_t* row,
                                                       size_t L, uint32_t top) {
        return g_glb(row, w & 0xffffu, top) | (g_glb(row + L, w >> 16, top) << 16);
    }
};

template <> struct Gather<4> {
    __device__ static __forceinline__ u32x2 lds(u32x2 w, const uint16_t* t, uint32_t top,
                                                int logW, int j) {
        u32x2 r;
        r.x = Gather<2>::lds(w.x, t, top, logW, j);
        r.y = Gather<2>::lds(w.y, t, top, logW, j + 2);
        return r;
    }
    __device__ static __forceinline__ u32x2 glb(u32x2 w, const uint16_t* row, size_t L,
                                                uint32_t top) {
        u32x2 r;
        r.x = Gather<2>::glb(w.x, row, L, top);
        r.y = Gather<2>::glb(w.y, row + 2 * L, L, top);
        return r;
    }
};

// One correction tile: band b, detectors [d0, d0 + weff), lines [n0, n1).
// Lanes own VEC adjacent detectors of one line; W / VEC lanes cover a strip
// line and the workgroup walks the lines UNROLL passes at a time, all loads
// of a pass issued before any gather so that many lines are in flight.
//
// LDS variant: the strip's LUT rows are first copied into `tile`
// (level-major, W * L entries) and every gather is an LDS read.
// Requirements (checked on the host): W = 2^logW, VEC | W, VEC | D, the
// image pointers aligned to 2*VEC bytes, W / VEC <= blockDim.x.
// dn and out may be the same buffer (in-place): every pixel is read and then
// written by the same lane, so they are deliberately not __restrict__.
template <int VEC, int UNROLL, bool NTH, bool LDS>
__device__ __forceinline__ void apply_tile(const uint16_t* dn, const uint16_t* __restrict__ lut,
                                           uint16_t* out, int64_t N, int D, int L,
                                           int logW, int b, int d0, int weff, int64_t n0,
                                           int64_t n1, uint16_t* tile, bool lut_vec) {
    typedef typename Px<VEC>::T T;
    const int W = 1 << logW;
    const int tid = threadIdx.x;
    const int nt = blockDim.x;
    const uint32_t top = (uint32_t)(L - 1);
    const uint16_t* strip_lut = lut + ((size_t)b * (size_t)D + (size_t)d0) * (size_t)L;

    if constexpr (LDS) {
        // Stage: lanes run along detectors (j fastest) so that one wave's
        // 16-bit LDS writes land in consecutive addresses.
        if (lut_vec) {
            const int items = (L >> 3) << logW;
            for (int it = tid; it < items; it += nt) {
                const int j = it & (W - 1);
                const int vc = it >> logW;
                if (j < weff) {
                    const u32x4 q = *(const u32x4*)(strip_lut + (size_t)j * (size_t)L + vc * 8);
                    uint16_t* dst = tile + ((vc * 8) << logW) + j;
                    dst[0] = (uint16_t)(q.x & 0xffffu);
                    dst[1 << logW] = (uint16_t)(q.x >> 16);
                    dst[2 << logW] = (uint16_t)(q.y & 0xffffu);
                    dst[3 << logW] = (uint16_t)(q.y >> 16);
                    dst[4 << logW] = (uint16_t)(q.z & 0xffffu);
                    dst[5 << logW] = (uint16_t)(q.z >> 16);
                    dst[6 << logW] = (uint16_t)(q.w & 0xffffu);
                    dst[7 << logW] = (uint16_t)(q.w >> 16);
                }
            }
        } else {
            const int items = L << logW;
            for (int it = tid; it < items; it += nt) {
                const int j = it & (W - 1);
                const int v = it >> logW;
                if (j < weff) tile[(v << logW) + j] = strip_lut[(size_t)j * (size_t)L + v];
            }
        }
        __syncthreads();
    }

    constexpr int LOGVEC = VEC == 1 ? 0 : (VEC == 2 ? 1 : 2);
    const int loglpr = logW - LOGVEC;  // lanes per strip line = W / VEC
    const int lane = tid & ((1 << loglpr) - 1);
    const int rpp = nt >> loglpr;  // lines per pass
    const int j = lane * VEC;
    if (j < weff) {
        const size_t Dz = (size_t)D;
        const size_t col = (size_t)d0 + (size_t)j;
        const size_t band0 = (size_t)b * (size_t)N;
        const uint16_t* lrow = strip_lut + (size_t)j * (size_t)L;
        for (int64_t n = n0 + (tid >> loglpr); n < n1; n += (int64_t)rpp * UNROLL) {
            T w[UNROLL];
#pragma unroll
            for (int u = 0; u < UNROLL; ++u) {
                const int64_t nn = n + (int64_t)u * rpp;
                if (nn < n1) {
                    w[u] = load_px<T, NTH>((const T*)(dn + (band0 + (size_t)nn) * Dz + col));
                }
            }
#pragma unroll
            for (int u = 0; u < UNROLL; ++u) {
                const int64_t nn = n + (int64_t)u * rpp;
                if (nn < n1) {
                    T r;
                    if constexpr (LDS) r = Gather<VEC>::lds(w[u], tile, top, logW, j);
                    else r = Gather<VEC>::glb(w[u], lrow, (size_t)L, top);
                    store_px<T, NTH>((T*)(out + (band0 + (size_t)nn) * Dz + col), r);
                }
            }
        }
    }
    if constexpr (LDS) __syncthreads();  // the tile may be restaged next
}

}  // namespace rc
