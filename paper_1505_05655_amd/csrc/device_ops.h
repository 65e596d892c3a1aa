// Device-side building blocks of the LUT build and correction kernels:
// the binary64 LUT entry, the XCD-aware tile order, and the correction tile
// with its three ways of reading the strip's LUT rows. Shared by the plain
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

template <int VEC> constexpr int log_vec() { return VEC == 1 ? 0 : (VEC == 2 ? 1 : 2); }

// Applies f(k, dn_k) to the VEC 16-bit DNs held in w and packs the results.
template <int VEC, typename F>
__device__ __forceinline__ typename Px<VEC>::T map_px(typename Px<VEC>::T w, F f) {
    if constexpr (VEC == 1) {
        return (unsigned short)f(0, (uint32_t)w);
    } else if constexpr (VEC == 2) {
        return f(0, w & 0xffffu) | (f(1, w >> 16) << 16);
    } else {
        u32x2 r;
        r.x = f(0, w.x & 0xffffu) | (f(1, w.x >> 16) << 16);
        r.y = f(2, w.y & 0xffffu) | (f(3, w.y >> 16) << 16);
        return r;
    }
}

// Streams lines [n0, n1) of detectors [col, col + VEC) of band `band0 / N`:
// UNROLL lines (rpp apart) are loaded before any is gathered and stored, so
// many loads are in flight per lane.
template <int VEC, int UNROLL, bool NTH, typename G>
__device__ __forceinline__ void stream_lines(const uint16_t* dn, uint16_t* out, size_t Dz,
                                             size_t band0, size_t col, int64_t first, int64_t n1,
                                             int rpp, G gather) {
    typedef typename Px<VEC>::T T;
    for (int64_t n = first; n < n1; n += (int64_t)rpp * UNROLL) {
        T w[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            const int64_t nn = n + (int64_t)u * rpp;
            if (nn < n1) w[u] = load_px<T, NTH>((const T*)(dn + (band0 + (size_t)nn) * Dz + col));
        }
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            const int64_t nn = n + (int64_t)u * rpp;
            if (nn < n1) {
                store_px<T, NTH>((T*)(out + (band0 + (size_t)nn) * Dz + col),
                                 map_px<VEC>(w[u], gather));
            }
        }
    }
}

// ---- the three LUT access modes -------------------------------------------------------

// Raw LDS strip, level-major: tile[v * W + j] is detector j's entry for level
// v. With W a multiple of 64 entries, the 32 lanes of a half-wave that own
// consecutive detector pairs read 32 different banks whatever the levels.
__device__ __forceinline__ uint32_t g_raw(const uint16_t* tile, uint32_t dnv, uint32_t top,
                                          int logW, int j) {
    const uint32_t v = dnv < top ? dnv : top;
    return tile[(v << logW) + j];
}

// Global LUT row (the L2 path).
__device__ __forceinline__ uint32_t g_glb(const uint16_t* row, uint32_t dnv, uint32_t top) {
    const uint32_t v = dnv < top ? dnv : top;
    return row[v];
}

// Packed LDS strip. Every LUT row is cut into blocks of 32 levels; a block is
// stored as its first entry (16-bit base) and the 31 steps between
// consecutive entries, each in {0, 1, 2, 3}, as two 32-bit bit-planes (bit i
// of `lo`/`hi` = low/high bit of step i). Entry v of the row is then
//   base[v / 32] + popcount(lo & m) + 2 * popcount(hi & m),  m = 2^(v % 32) - 1,
// exactly. That is 2.5 bits per entry instead of 16, so strips 6.4x wider fit
// in LDS. Rows with a negative step or a step above 3 cannot be packed; the
// tile then falls back to global gathers. Layout: planes [NB][W] (u32x2)
// followed by bases [NB][W] (u16), detector j of the strip at position
// p = (j % VEC) * (W / VEC) + j / VEC, so the lanes of a wave read
// consecutive 8-byte plane words for each of their VEC pixels.
__device__ __forceinline__ uint32_t g_packed(const u32x2* planes, const uint16_t* bases,
                                             uint32_t dnv, uint32_t top, int logW, int p) {
    const uint32_t v = dnv < top ? dnv : top;
    const int idx = (int)((v >> 5) << logW) + p;
    const u32x2 q = planes[idx];
    const uint32_t m = (1u << (v & 31u)) - 1u;
    return (uint32_t)bases[idx] + (uint32_t)__builtin_popcount(q.x & m) +
           2u * (uint32_t)__builtin_popcount(q.y & m);
}

// Bytes of LDS a packed strip of W detectors needs for L levels.
__host__ __device__ constexpr size_t packed_lds_bytes(int W, int L) {
    return (size_t)((L + 31) / 32) * (size_t)W * 10;
}

enum TileMode { kRaw = 0, kGlobal = 1, kPacked = 2 };

// One correction tile: band b, detectors [d0, d0 + weff), lines [n0, n1).
// Lanes own VEC adjacent detectors of one line; W / VEC lanes cover a strip
// line and the workgroup walks the lines. Requirements (checked on the host):
// W = 2^logW, VEC | W, VEC | D, image pointers aligned to 2*VEC bytes,
// W / VEC <= blockDim.x, and the LDS size of the mode. dn and out may be the
// same buffer (in place): every pixel is read and then written by the same
// lane, so they are deliberately not __restrict__.
template <int VEC, int UNROLL, bool NTH, int MODE>
__device__ __forceinline__ void apply_tile(const uint16_t* dn, const uint16_t* __restrict__ lut,
                                           uint16_t* out, int64_t N, int D, int L, int logW,
                                           int b, int d0, int weff, int64_t n0, int64_t n1,
                                           void* smem, bool lut_vec) {
    constexpr int LOGVEC = log_vec<VEC>();
    const int W = 1 << logW;
    const int tid = threadIdx.x;
    const int nt = blockDim.x;
    const uint32_t top = (uint32_t)(L - 1);
    const size_t Lz = (size_t)L;
    const uint16_t* strip_lut = lut + ((size_t)b * (size_t)D + (size_t)d0) * Lz;
    const int logq = logW - LOGVEC;  // lanes per strip line = W / VEC
    const int lane = tid & ((1 << logq) - 1);
    const int rpp = nt >> logq;      // lines per pass
    const int j = lane * VEC;
    const size_t band0 = (size_t)b * (size_t)N;
    const size_t col = (size_t)d0 + (size_t)j;
    const int64_t first = n0 + (tid >> logq);

    if constexpr (MODE == kRaw) {
        uint16_t* tile = (uint16_t*)smem;
        // Stage: lanes run along detectors (j fastest) so that one wave's
        // 16-bit LDS writes land in consecutive addresses.
        if (lut_vec) {
            const int items = (L >> 3) << logW;
            for (int it = tid; it < items; it += nt) {
                const int jj = it & (W - 1);
                const int vc = it >> logW;
                if (jj < weff) {
                    const u32x4 q = *(const u32x4*)(strip_lut + (size_t)jj * Lz + vc * 8);
                    uint16_t* dst = tile + ((vc * 8) << logW) + jj;
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
                const int jj = it & (W - 1);
                const int v = it >> logW;
                if (jj < weff) tile[(v << logW) + jj] = strip_lut[(size_t)jj * Lz + v];
            }
        }
        __syncthreads();
        if (j < weff) {
            stream_lines<VEC, UNROLL, NTH>(
                dn, out, (size_t)D, band0, col, first, n1, rpp,
                [&](int k, uint32_t d) { return g_raw(tile, d, top, logW, j + k); });
        }
        __syncthreads();  // the tile may be restaged next
    } else if constexpr (MODE == kGlobal) {
        if (j < weff) {
            const uint16_t* lrow = strip_lut + (size_t)j * Lz;
            stream_lines<VEC, UNROLL, NTH>(
                dn, out, (size_t)D, band0, col, first, n1, rpp,
                [&](int k, uint32_t d) { return g_glb(lrow + (size_t)k * Lz, d, top); });
        }
    } else {
        const int NB = (L + 31) >> 5;
        u32x2* planes = (u32x2*)smem;
        uint16_t* bases = (uint16_t*)(planes + (size_t)NB * W);
        // Stage: item = (detector jj, block) with blocks fastest, so a wave
        // reads long contiguous runs of one LUT row.
        int bad = 0;
        const int items = weff * NB;
        for (int it = tid; it < items; it += nt) {
            const int jj = it / NB;
            const int blk = it - jj * NB;
            const uint16_t* src = strip_lut + (size_t)jj * Lz + (size_t)blk * 32;
            const int cnt = min(32, L - blk * 32);
            uint32_t e[32];
            if (lut_vec && cnt == 32) {
#pragma unroll
                for (int q4 = 0; q4 < 4; ++q4) {
                    const u32x4 q = *(const u32x4*)(src + q4 * 8);
                    e[q4 * 8 + 0] = q.x & 0xffffu;
                    e[q4 * 8 + 1] = q.x >> 16;
                    e[q4 * 8 + 2] = q.y & 0xffffu;
                    e[q4 * 8 + 3] = q.y >> 16;
                    e[q4 * 8 + 4] = q.z & 0xffffu;
                    e[q4 * 8 + 5] = q.z >> 16;
                    e[q4 * 8 + 6] = q.w & 0xffffu;
                    e[q4 * 8 + 7] = q.w >> 16;
                }
            } else {
#pragma unroll
                for (int i = 0; i < 32; ++i) e[i] = i < cnt ? src[i] : 0u;
            }
            uint32_t lo = 0, hi = 0;
#pragma unroll
            for (int i = 0; i < 31; ++i) {
                if (i + 1 < cnt) {
                    const uint32_t step = e[i + 1] - e[i];  // wraps when negative
                    bad |= step > 3u;
                    lo |= (step & 1u) << i;
                    hi |= ((step >> 1) & 1u) << i;
                }
            }
            const int p = ((jj & (VEC - 1)) << logq) + (jj >> LOGVEC);
            u32x2 pl;
            pl.x = lo;
            pl.y = hi;
            planes[blk * W + p] = pl;
            bases[blk * W + p] = (uint16_t)e[0];
        }
        bad = __syncthreads_or(bad);
        if (j < weff) {
            if (!bad) {
                stream_lines<VEC, UNROLL, NTH>(
                    dn, out, (size_t)D, band0, col, first, n1, rpp, [&](int k, uint32_t d) {
                        return g_packed(planes, bases, d, top, logW, (k << logq) + lane);
                    });
            } else {
                const uint16_t* lrow = strip_lut + (size_t)j * Lz;
                stream_lines<VEC, UNROLL, NTH>(
                    dn, out, (size_t)D, band0, col, first, n1, rpp,
                    [&](int k, uint32_t d) { return g_glb(lrow + (size_t)k * Lz, d, top); });
            }
        }
        __syncthreads();  // the tile may be restaged next
    }
}

}  // namespace rc
