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
// Horner from the cubic coefficient down, one rounding per operation, then
// round half away from zero and clamp to [0, L-1]. `lim` is (double)L.
// The rounding and clamp are done as: c = min(max(acc, 0), L) in binary64
// (maxNum sends NaN to 0, -Inf and every negative to 0, +Inf to L), then
// r = trunc(c + h) with h = 0.5 - 2^-54 (the double just below 1/2), then
// min(r, L-1). For 0 <= c < 2^52, trunc(fl(c + h)) is round-half-away(c):
// if frac(c) >= 1/2 the exact sum is at least n - 2^-54 for n = ceil(c), and
// it only falls below n when c = n - 1/2, where n - 2^-54 rounds up to n
// (a tie to even at n = 1, nearer n above); if frac(c) < 1/2 the exact sum
// is at most floor(c) + 1 - ulp(c) - 2^-54, more than half an ulp below
// floor(c) + 1, so it cannot round up to it. With plain 1/2 instead of h,
// c = 1/2 - 2^-54 would round to 1.
__device__ __forceinline__ uint32_t lut_entry(double a0, double a1, double a2, double a3, int v,
                                              double lim) {
    const double x = (double)v;
    double acc = a3;
    acc = acc * x;
    acc = acc + a2;
    acc = acc * x;
    acc = acc + a1;
    acc = acc * x;
    acc = acc + a0;
    const double c = __builtin_fmin(__builtin_fmax(acc, 0.0), lim);
    const uint32_t r = (uint32_t)(c + 0x1.fffffffffffffp-2);
    const uint32_t top = (uint32_t)lim - 1u;
    return r < top ? r : top;
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

// VEC pixels of one line held by one lane.
template <int VEC> struct Px;
template <> struct Px<1> { typedef unsigned short T; };
template <> struct Px<2> { typedef unsigned int T; };
template <> struct Px<4> { typedef u32x2 T; };
template <> struct Px<8> { typedef u32x4 T; };

template <int VEC> constexpr int log_vec() {
    return VEC == 1 ? 0 : (VEC == 2 ? 1 : (VEC == 4 ? 2 : 3));
}

// Applies f(k, dn_k) to the VEC 16-bit DNs held in w and packs the results.
template <int VEC, typename F>
__device__ __forceinline__ typename Px<VEC>::T map_px(typename Px<VEC>::T w, F f) {
    if constexpr (VEC == 1) {
        return (unsigned short)f(0, (uint32_t)w);
    } else if constexpr (VEC == 2) {
        return f(0, w & 0xffffu) | (f(1, w >> 16) << 16);
    } else if constexpr (VEC == 4) {
        u32x2 r;
        r.x = f(0, w.x & 0xffffu) | (f(1, w.x >> 16) << 16);
        r.y = f(2, w.y & 0xffffu) | (f(3, w.y >> 16) << 16);
        return r;
    } else {
        u32x4 r;
        r.x = f(0, w.x & 0xffffu) | (f(1, w.x >> 16) << 16);
        r.y = f(2, w.y & 0xffffu) | (f(3, w.y >> 16) << 16);
        r.z = f(4, w.z & 0xffffu) | (f(5, w.z >> 16) << 16);
        r.w = f(6, w.w & 0xffffu) | (f(7, w.w >> 16) << 16);
        return r;
    }
}

// Raw buffer resource over `bytes` bytes from `base` (gfx9-family word 3:
// untyped 32-bit data). Buffer loads past `bytes` return 0 and stores past
// it are dropped, so a tile's last partial pass needs no per-line guard.
constexpr int kRsrcWord3 = 0x00020000;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes,
                                             kRsrcWord3);
}

typedef int i32x2 __attribute__((ext_vector_type(2)));
typedef int i32x4 __attribute__((ext_vector_type(4)));

// Image cache policy NT -> the cache-policy bits of the buffer loads and
// stores (gfx950: bit 0 sc0, bit 1 nt, bit 4 sc1):
//   0 default,  1 nt loads and stores,  2 nt stores,
//   3 sc0 loads + nt stores,  4 sc1 loads + nt stores,  5 sc0 loads.
constexpr int kPolicies = 6;
constexpr int ld_aux(int nt) { return nt == 1 ? 2 : (nt == 3 || nt == 5 ? 1 : (nt == 4 ? 16 : 0)); }
constexpr int st_aux(int nt) { return nt >= 1 && nt <= 4 ? 2 : 0; }

// VEC pixels of one line through a buffer resource: per-lane byte offset
// `vo` (VGPR) plus a wave-uniform line offset `so` (SGPR); NT is the image
// cache policy above.
template <int VEC, int NT> struct Buf;
template <int NT> struct Buf<1, NT> {
    static __device__ __forceinline__ unsigned short ld(__amdgpu_buffer_rsrc_t r, uint32_t vo,
                                                        uint32_t so) {
        return (unsigned short)__builtin_amdgcn_raw_buffer_load_b16(r, (int)vo, (int)so,
                                                                    ld_aux(NT));
    }
    static __device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so,
                                              unsigned short v) {
        __builtin_amdgcn_raw_buffer_store_b16((short)v, r, (int)vo, (int)so, st_aux(NT));
    }
};
template <int NT> struct Buf<2, NT> {
    static __device__ __forceinline__ unsigned int ld(__amdgpu_buffer_rsrc_t r, uint32_t vo,
                                                      uint32_t so) {
        return (unsigned int)__builtin_amdgcn_raw_buffer_load_b32(r, (int)vo, (int)so,
                                                                  ld_aux(NT));
    }
    static __device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so,
                                              unsigned int v) {
        __builtin_amdgcn_raw_buffer_store_b32((int)v, r, (int)vo, (int)so, st_aux(NT));
    }
};
template <int NT> struct Buf<4, NT> {
    static __device__ __forceinline__ u32x2 ld(__amdgpu_buffer_rsrc_t r, uint32_t vo,
                                               uint32_t so) {
        return (u32x2)__builtin_amdgcn_raw_buffer_load_b64(r, (int)vo, (int)so, ld_aux(NT));
    }
    static __device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so,
                                              u32x2 v) {
        __builtin_amdgcn_raw_buffer_store_b64((i32x2)v, r, (int)vo, (int)so, st_aux(NT));
    }
};
template <int NT> struct Buf<8, NT> {
    static __device__ __forceinline__ u32x4 ld(__amdgpu_buffer_rsrc_t r, uint32_t vo,
                                               uint32_t so) {
        return (u32x4)__builtin_amdgcn_raw_buffer_load_b128(r, (int)vo, (int)so, ld_aux(NT));
    }
    // A store of more than 8 bytes reads its data registers after issue; the
    // compiler only keeps the next VALU off them when soffset is not a
    // register (measured on gfx950: with the line offset in an SGPR, the loop
    // counter update right after the store overwrote its first dword). The
    // whole offset therefore goes in the VGPR, soffset is the constant 0.
    static __device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so,
                                              u32x4 v) {
        __builtin_amdgcn_raw_buffer_store_b128((i32x4)v, r, (int)(vo + so), 0, st_aux(NT));
    }
};

// Streams `passes` passes over a tile's lines. In each pass a lane handles
// its VEC pixels of UNROLL lines (line_stride bytes apart); consecutive
// passes start pass_adv bytes apart (0: UNROLL * line_stride, contiguous
// lines; a multiple of it when a tile takes every k-th pass). Software
// pipelined with two register sets used alternately: the loads of pass k+1
// are issued before pass k is gathered and stored, so a wave's memory
// latency overlaps its own gather work (no register copies between the sets,
// which would force a wait on the prefetched loads). The prefetch past the
// last pass falls outside the buffer range (loads of 0); offsets stay below
// 2^31 because tiles are sized with two passes of slack.
template <int VEC, int UNROLL, int NT, typename G>
__device__ __forceinline__ void stream_lines(__amdgpu_buffer_rsrc_t rin,
                                             __amdgpu_buffer_rsrc_t rout, uint32_t vo,
                                             uint32_t line_stride, int passes, G gather,
                                             uint32_t pass_adv = 0) {
    typedef typename Px<VEC>::T T;
    const uint32_t pass_bytes = pass_adv ? pass_adv : UNROLL * line_stride;
    T a[UNROLL], b[UNROLL];
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) a[u] = Buf<VEC, NT>::ld(rin, vo, u * line_stride);
    uint32_t so = 0;  // wave-uniform line offset of the current pass
    for (int k = 0; k < passes; k += 2) {
        so = __builtin_amdgcn_readfirstlane(so);
#pragma unroll
        for (int u = 0; u < UNROLL; ++u)
            b[u] = Buf<VEC, NT>::ld(rin, vo, so + pass_bytes + u * line_stride);
#pragma unroll
        for (int u = 0; u < UNROLL; ++u)
            Buf<VEC, NT>::st(rout, vo, so + u * line_stride, map_px<VEC>(a[u], gather));
        if (k + 1 >= passes) break;
        so += pass_bytes;
#pragma unroll
        for (int u = 0; u < UNROLL; ++u)
            a[u] = Buf<VEC, NT>::ld(rin, vo, so + pass_bytes + u * line_stride);
#pragma unroll
        for (int u = 0; u < UNROLL; ++u)
            Buf<VEC, NT>::st(rout, vo, so + u * line_stride, map_px<VEC>(b[u], gather));
        so += pass_bytes;
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

// ---- dense LDS strip: one bit per step -------------------------------------------------
//
// A LUT row is cut into blocks of 64 levels. Within block `blk` the entries
// e_0..e_63 are stored as an unclamped staircase U_0..U_63 with
// clamp(U_i, 0, L-1) = e_i:
//   U_i = U_0 + s*i + sum_{t<i} b_t,   s in {0, 1},  b_t in {0, 1},
// i.e. each step U_{t+1} - U_t is s or s + 1. Where the row saturates
// (entries 0 before the first positive one, entries L-1 from the first L-1
// on) the staircase goes on below 0 / above L-1 in steps of s + 1 and the
// clamp restores the entries. The encoder takes s = max(0, largest step -
// 1), so a block whose only unsaturated step is 2 (a jump into or out of a
// saturated run) still fits.
//
// Stored form, chosen so that the decode is additive and needs no masks:
//   plane z: bit 63 - t = 1 - b_t (t = 0..62), bit 0 = s;
//   header H (int16) = U_0 + B - 63 - 64*(s+1)*blk - s,  B = sum_t b_t.
// Shifting z left by i keeps bits 0..63-i, i.e. the complemented steps
// t >= i and bit 0, so popcount(z << i) = (63 - i) - sum_{t>=i} b_t + s and,
// with m = s + 1 and level v = 64*blk + i,
//   U = H + m*v + popcount(z << (v mod 64))      (m*v = v << s),
// exactly. |H| < 16448 for L <= 8192, so H never equals kDenseBad, the
// header that marks a block the dense form cannot hold. 80 bits per 64
// entries (1.25 bits per entry): a 4096-level strip of 256 detectors fits
// 160 KiB. Encodable blocks: non-decreasing, with the steps between
// unsaturated entries within {s, s+1}, s <= 1 (calibration LUTs: gains
// below 2); other rows make the tile gather from the global LUT.
// Layout: planes [NB][W] (64-bit) from byte 0, then headers [NB][W] (int16)
// from byte NB * W * 8; detector j of the strip at position p = (j % VEC) *
// (W / VEC) + j / VEC, as the packed strip. A lane keeps 8p and its header
// base NB*W*8 + 2p, so each of the two addresses of a level is one shift-add
// of the block index. Requires L <= kDenseMaxLevels = 8192 (header range).
constexpr int16_t kDenseBad = -32768;

__host__ __device__ constexpr size_t dense_lds_bytes(int W, int L) {
    return (size_t)((L + 63) / 64) * (size_t)W * 10;
}

// LDS addressed from byte 0: the correction kernels have no static LDS, so
// their dynamic LDS starts at 0 (prepare_apply_kernels and
// prepare_batch_kernel check it on the host and refuse otherwise); with the
// base a known constant no address needs an add for it.
typedef __attribute__((address_space(3))) const uint64_t lds_u64;
typedef __attribute__((address_space(3))) const int16_t lds_i16;

// med3(x, 0, hi) in one instruction (the compiler forms it only for
// constant bounds); hi is wave-uniform.
__device__ __forceinline__ uint32_t clamp0(int x, int hi) {
    int r;
    asm("v_med3_i32 %0, %1, 0, %2" : "=v"(r) : "v"(x), "s"(hi));
    return (uint32_t)r;
}

// popcount(x) + acc in one instruction (the compiler would otherwise sum
// two popcounts with a separate three-way add).
__device__ __forceinline__ int bcnt_acc(uint32_t x, int acc) {
    int r;
    asm("v_bcnt_u32_b32 %0, %1, %2" : "=v"(r) : "v"(x), "v"(acc));
    return r;
}

// p8 = 8p, h2 = NB*W*8 + 2p (the lane's position p in the plane and header
// arrays, in bytes from the start of LDS).
__device__ __forceinline__ uint32_t g_dense(uint32_t dnv, uint32_t top, int logW, uint32_t p8,
                                            uint32_t h2) {
    const uint32_t v = dnv < top ? dnv : top;
    const uint32_t blk = v >> 6;
    const uint64_t z = *(lds_u64*)(uintptr_t)((blk << (logW + 3)) + p8);
    const int h = *(lds_i16*)(uintptr_t)((blk << (logW + 1)) + h2);
    const uint64_t sh = z << (v & 63u);
    int u = (int)(v << ((uint32_t)z & 1u)) + h;
    u = bcnt_acc((uint32_t)(sh >> 32), u);
    u = bcnt_acc((uint32_t)sh, u);
    return clamp0(u, (int)top);
}

// As g_dense, for a strip with blocks the dense form cannot hold: a level of
// such a block (header kDenseBad) reads the LUT row in global memory.
__device__ __forceinline__ uint32_t g_dense_checked(uint32_t dnv, uint32_t top, int logW,
                                                    uint32_t p8, uint32_t h2,
                                                    const uint16_t* row) {
    const uint32_t v = dnv < top ? dnv : top;
    const uint32_t blk = v >> 6;
    const int h = *(lds_i16*)(uintptr_t)((blk << (logW + 1)) + h2);
    if (h == (int)kDenseBad) return row[v];
    const uint64_t z = *(lds_u64*)(uintptr_t)((blk << (logW + 3)) + p8);
    const uint64_t sh = z << (v & 63u);
    int u = (int)(v << ((uint32_t)z & 1u)) + h;
    u = bcnt_acc((uint32_t)(sh >> 32), u);
    u = bcnt_acc((uint32_t)sh, u);
    return clamp0(u, (int)top);
}

// Encodes block `blk` (n entries, 1..64) of a LUT row: e holds the entries
// two per word (entry 2k in the low half of e[k]). Returns false when the
// block is not encodable.
__device__ __forceinline__ bool dense_encode(const uint32_t (&e)[32], int n, uint32_t top, int blk,
                                             uint64_t* plane, int16_t* head) {
    auto at = [&](int i) -> int { return (int)((e[i >> 1] >> ((i & 1) * 16)) & 0xffffu); };
    // Pass 1: smallest and largest step.
    int mn = 1 << 20, mx = -(1 << 20);
#pragma unroll
    for (int t = 0; t < 63; ++t) {
        if (t + 1 < n) {
            const int st = at(t + 1) - at(t);
            mn = min(mn, st);
            mx = max(mx, st);
        }
    }
    if (n > 1 && mn < 0) return false;  // decreasing somewhere
    const int e0 = at(0), elast = at(n - 1);
    // b: bit t+1 = b_t (the step-minus-slope bits, t = 0..62).
    uint32_t lo = 0, hi = 0;
    int s = 0, u0 = 0;
    if (n == 1 || e0 == (int)top || elast == 0) {
        // Constant (a single entry, all L-1, or all 0 in a non-decreasing block).
        u0 = e0;
    } else if (e0 != 0 && elast != (int)top) {
        // No saturated entry (non-decreasing, 0 < e0, e_last < L-1). Any
        // s in [mx - 1, mn] holds the steps; the largest keeps s <= 1 for
        // the most blocks.
        s = max(0, mx - 1);
        if (s > 1 || mn < s) return false;
        u0 = e0;
#pragma unroll
        for (int t = 0; t < 63; ++t) {
            if (t + 1 < n) {
                const uint32_t b = (uint32_t)(at(t + 1) - at(t) - s);
                if (t + 1 < 32) lo |= b << (t + 1);
                else hi |= b << (t + 1 - 32);
            }
        }
    } else {
        // A saturation transition inside the block. Steps between two
        // unsaturated entries (the step out of a run of 0 and into a run of
        // L-1 included) set the slope; steps inside a saturated run are s + 1.
        int smin = 1 << 20, smax = -(1 << 20), first = n;
#pragma unroll
        for (int t = 0; t < 63; ++t) {
            if (t + 1 < n) {
                const int a = at(t), b = at(t + 1);
                if (b != 0 && a != (int)top) {
                    smin = min(smin, b - a);
                    smax = max(smax, b - a);
                }
                if (a == 0 && b != 0 && first == n) first = t + 1;
            }
        }
        s = max(0, smax - 1);
        if (s > 1 || smin < s) return false;
        // U_{first-1} = 0 when the block opens with a run of 0.
        u0 = e0 != 0 ? e0 : -(s + 1) * (first - 1);
#pragma unroll
        for (int t = 0; t < 63; ++t) {
            if (t + 1 < n) {
                const int a = at(t), b = at(t + 1);
                const uint32_t bit = (b != 0 && a != (int)top) ? (uint32_t)(b - a - s) : 1u;
                if (t + 1 < 32) lo |= bit << (t + 1);
                else hi |= bit << (t + 1 - 32);
            }
        }
    }
    const uint64_t bits = ((uint64_t)hi << 32) | lo;
    // Bit t+1 of `bits` -> bit 63-t, complemented; bit 0 <- s.
    const uint64_t z = (~(__builtin_bitreverse64(bits) << 1) & ~(uint64_t)1) | (uint64_t)s;
    const int H = u0 + __builtin_popcountll(bits) - 63 - 64 * (s + 1) * blk - s;
    if (H <= (int)kDenseBad || H > 32767) return false;
    *plane = z;
    *head = (int16_t)H;
    return true;
}

// Encodes block `blk` of LUT row `row` (L levels) into *plane and *head; a
// block that does not fit the dense form gets the header kDenseBad.
__device__ __forceinline__ void dense_encode_row_block(const uint16_t* row, int L, int blk,
                                                      bool vec16, uint64_t* plane, int16_t* head) {
    const uint16_t* src = row + (size_t)blk * 64;
    const int cnt = min(64, L - blk * 64);
    uint32_t e[32];
    if (vec16 && cnt == 64) {
#pragma unroll
        for (int q4 = 0; q4 < 8; ++q4) {
            const u32x4 w = *(const u32x4*)(src + q4 * 8);
            e[q4 * 4 + 0] = w.x;
            e[q4 * 4 + 1] = w.y;
            e[q4 * 4 + 2] = w.z;
            e[q4 * 4 + 3] = w.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < 32; ++k) {
            const uint32_t a = 2 * k < cnt ? src[2 * k] : 0u;
            const uint32_t c = 2 * k + 1 < cnt ? src[2 * k + 1] : 0u;
            e[k] = a | (c << 16);
        }
    }
    uint64_t pl = 0;
    int16_t hd = kDenseBad;
    if (!dense_encode(e, cnt, (uint32_t)(L - 1), blk, &pl, &hd)) hd = kDenseBad;
    *plane = pl;
    *head = hd;
}

// Workgroup-wide OR of `flag` for a dense strip, without static LDS: a
// wave with the flag set writes kDenseBad (a header no encodable block has)
// over the first header; the tile then does not decode the strip. Call
// after every thread has staged; every thread returns the same value.
__device__ __forceinline__ int dense_any(int flag, int16_t* heads) {
    __syncthreads();
    if (__any(flag) && (threadIdx.x & 63) == 0) heads[0] = kDenseBad;
    __syncthreads();
    return (int)(heads[0] == kDenseBad);
}

enum TileMode { kRaw = 0, kGlobal = 1, kPacked = 2, kDense = 3 };

// Workgroup-wide OR of `flag` for a packed strip, without static LDS (a
// static word would push two 80 KiB tiles over a CU's 160 KiB). The word is
// bit 31 of the first plane word: a block has 31 steps, so staging leaves
// bit 31 clear and the gather masks never reach it. Call after every thread
// has staged (planes[0] is always written: detector 0, block 0); every
// thread returns the same value.
__device__ __forceinline__ int packed_any(int flag, u32x2* planes) {
    __syncthreads();
    if (__any(flag) && (threadIdx.x & 63) == 0)
        atomicOr((unsigned int*)planes, 0x80000000u);
    __syncthreads();
    return (int)(*(const unsigned int*)planes >> 31);
}

// One correction tile: band b, detectors [d0, d0 + weff), lines [n0, n1).
// Lanes own VEC adjacent detectors of one line; q consecutive threads cover
// a line of the strip and the workgroup walks floor(blockDim.x / q) lines at
// a time. q = W / VEC (`dense` false: a wave covers whole line segments when
// q divides 64, lanes past a narrower strip idle) or weff / VEC (`dense`
// true: no idle lanes inside a wave). Requirements (checked on the host): W = 2^logW >= weff, VEC | W,
// VEC | weff, VEC | d0, VEC | D, image pointers aligned to 2*VEC bytes,
// W / VEC <= blockDim.x, and the LDS size of the mode for W detectors. dn and
// out may be the same buffer (in place): every pixel is read and then written
// by the same lane, so they are deliberately not __restrict__.
// LANE_ENCODE: the dense mode may encode its strip from the global LUT
// (false: the caller always passes a pre-encoded strip, and the encoder is
// not compiled in).
template <int VEC, int UNROLL, int NT, int MODE, bool LANE_ENCODE = true>
__device__ __forceinline__ void apply_tile(const uint16_t* dn, const uint16_t* __restrict__ lut,
                                           uint16_t* out, int64_t N, int D, int L, int logW,
                                           int b, int d0, int weff, int64_t n0, int64_t n1,
                                           void* smem, bool lut_vec, bool dense,
                                           const uint64_t* pre_planes = nullptr,
                                           const int16_t* pre_heads = nullptr, int ci = 0,
                                           int ck = 1, int nst = 0) {
    constexpr int LOGVEC = log_vec<VEC>();
    const int W = 1 << logW;
    const int tid = threadIdx.x;
    const int nt = blockDim.x;
    const uint32_t top = (uint32_t)(L - 1);
    const size_t Lz = (size_t)L;
    const uint16_t* strip_lut = lut + ((size_t)b * (size_t)D + (size_t)d0) * Lz;
    const int logq = logW - LOGVEC;  // LDS positions per VEC slot = W / VEC
    const int q = dense ? (weff >> LOGVEC) : (1 << logq);  // lanes per strip line
    const int row = tid / q;         // this thread's line within a pass
    const int lane = tid - row * q;
    // Lines per pass, from the nst streaming threads (0: all of them).
    // Wave-uniform (the compiler cannot prove it through the division and
    // would otherwise wrap every buffer access in a waterfall loop).
    const int rpp = __builtin_amdgcn_readfirstlane((nst ? nst : nt) / q);
    // Threads past the last whole line, or past the strip, only stage.
    const bool streams = row < rpp && lane * VEC < weff;
    const int j = lane * VEC;
    // The tile's image bytes as buffer resources: line n0, detector d0 is at
    // byte 0; the range ends after the tile's last pixel.
    const size_t tile0 = ((size_t)b * (size_t)N + (size_t)n0) * (size_t)D + (size_t)d0;
    const uint32_t span = (uint32_t)((((size_t)(n1 - n0) - 1) * (size_t)D + (size_t)weff) * 2);
    const __amdgpu_buffer_rsrc_t rin = make_rsrc(dn + tile0, span);
    const __amdgpu_buffer_rsrc_t rout = make_rsrc(out + tile0, span);
    // Passes of rpp x UNROLL lines over [n0, n1); the tile takes passes ci,
    // ci + ck, ci + 2 ck, ... (ck = 1: all of them).
    const uint32_t line_stride = (uint32_t)rpp * (uint32_t)D * 2u;
    const uint32_t pass_bytes = UNROLL * line_stride;
    const uint32_t pass_adv = pass_bytes * (uint32_t)ck;
    const uint32_t vo = (uint32_t)(((size_t)row * (size_t)D + (size_t)j) * 2) +
                        (uint32_t)ci * pass_bytes;
    const int all_passes =
        (int)((n1 - n0 + (int64_t)rpp * UNROLL - 1) / ((int64_t)rpp * UNROLL));
    const int passes = ci < all_passes ? (all_passes - ci + ck - 1) / ck : 0;

    if constexpr (MODE == kRaw) {
        uint16_t* tile = (uint16_t*)smem;
        // Stage: lanes run along detectors (j fastest) so that one wave's
        // 16-bit LDS writes land in consecutive addresses.
        if (lut_vec) {
            // Rounds of SU items per thread, loads first (latency overlap).
            constexpr int SU = 8;
            const int items = (L >> 3) << logW;
            for (int it0 = tid; it0 < items; it0 += nt * SU) {
                u32x4 qv[SU];
#pragma unroll
                for (int s = 0; s < SU; ++s) {
                    const int it = it0 + s * nt;
                    const int jj = it & (W - 1);
                    qv[s] = u32x4{0u, 0u, 0u, 0u};
                    if (it < items && jj < weff) {
                        qv[s] = *(const u32x4*)(strip_lut + (size_t)jj * Lz + (it >> logW) * 8);
                    }
                }
#pragma unroll
                for (int s = 0; s < SU; ++s) {
                    const int it = it0 + s * nt;
                    const int jj = it & (W - 1);
                    if (it < items && jj < weff) {
                        const u32x4 q = qv[s];
                        uint16_t* dst = tile + (((it >> logW) * 8) << logW) + jj;
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
        if (streams) {
            stream_lines<VEC, UNROLL, NT>(
                rin, rout, vo, line_stride, passes,
                [&](int k, uint32_t d) { return g_raw(tile, d, top, logW, j + k); }, pass_adv);
        }
        __syncthreads();  // the tile may be restaged next
    } else if constexpr (MODE == kGlobal) {
        if (streams) {
            const uint16_t* lrow = strip_lut + (size_t)j * Lz;
            stream_lines<VEC, UNROLL, NT>(
                rin, rout, vo, line_stride, passes,
                [&](int k, uint32_t d) { return g_glb(lrow + (size_t)k * Lz, d, top); }, pass_adv);
        }
    } else if constexpr (MODE == kDense) {
        const int NB = (L + 63) >> 6;
        const uint32_t hb = (uint32_t)NB << (logW + 3);  // header array, bytes from LDS start
        uint64_t* planes = (uint64_t*)smem;
        int16_t* heads = (int16_t*)((unsigned char*)smem + hb);
        int bad = 0;
        if (pre_planes) {
            // Stage the blocks k_dense_encode wrote ([band][block][detector]):
            // consecutive threads read consecutive detectors of one block.
            const int items = NB * weff;
            const size_t row0 = (size_t)b * (size_t)NB * (size_t)D + (size_t)d0;
            for (int it = tid; it < items; it += nt) {
                const int blk = it / weff;
                const int jj = it - blk * weff;
                const size_t g = row0 + (size_t)blk * (size_t)D + (size_t)jj;
                const int16_t hd = pre_heads[g];
                const int p = ((jj & (VEC - 1)) << logq) + (jj >> LOGVEC);
                bad |= (int)(hd == kDenseBad);
                planes[(blk << logW) + p] = pre_planes[g];
                heads[(blk << logW) + p] = hd;
            }
        }
        // Stage: one lane encodes one block (detector jj, 64 levels); a wave
        // covers 64 consecutive LDS positions of one block index, so its
        // plane and header writes are consecutive words.
        const int units = (!LANE_ENCODE || pre_planes) ? 0 : NB << logW;
        for (int u = tid; LANE_ENCODE && u < units; u += nt) {
            const int blk = u >> logW;
            const int p = u & (W - 1);
            const int jj = ((p & ((1 << logq) - 1)) << LOGVEC) + (p >> logq);
            if (jj >= weff) continue;
            const uint16_t* src = strip_lut + (size_t)jj * Lz + (size_t)blk * 64;
            const int cnt = min(64, L - blk * 64);
            uint32_t e[32];
            if (lut_vec && cnt == 64) {
#pragma unroll
                for (int q4 = 0; q4 < 8; ++q4) {
                    const u32x4 w = *(const u32x4*)(src + q4 * 8);
                    e[q4 * 4 + 0] = w.x;
                    e[q4 * 4 + 1] = w.y;
                    e[q4 * 4 + 2] = w.z;
                    e[q4 * 4 + 3] = w.w;
                }
            } else {
#pragma unroll
                for (int k = 0; k < 32; ++k) {
                    const uint32_t a = 2 * k < cnt ? src[2 * k] : 0u;
                    const uint32_t b = 2 * k + 1 < cnt ? src[2 * k + 1] : 0u;
                    e[k] = a | (b << 16);
                }
            }
            uint64_t pl = 0;
            int16_t hd = kDenseBad;
            if (!dense_encode(e, cnt, top, blk, &pl, &hd)) bad = 1;
            planes[u] = pl;
            heads[u] = hd;
        }
        bad = dense_any(bad, heads);
        if (streams) {
            if (!bad) {
                stream_lines<VEC, UNROLL, NT>(
                    rin, rout, vo, line_stride, passes, [&](int k, uint32_t d) {
                        const uint32_t p = (uint32_t)((k << logq) + lane);
                        return g_dense(d, top, logW, p * 8u, hb + p * 2u);
                    }, pass_adv);
            } else {
                // Some blocks of the strip (or, with the flag's word, block 0
                // of its first position) are not held in dense form: their
                // levels read the global LUT row, every other level decodes.
                const uint16_t* lrow = strip_lut + (size_t)j * Lz;
                stream_lines<VEC, UNROLL, NT>(
                    rin, rout, vo, line_stride, passes, [&](int k, uint32_t d) {
                        const uint32_t p = (uint32_t)((k << logq) + lane);
                        return g_dense_checked(d, top, logW, p * 8u, hb + p * 2u,
                                               lrow + (size_t)k * Lz);
                    }, pass_adv);
            }
        }
        __syncthreads();  // the tile may be restaged next
    } else {
        const int NB = (L + 31) >> 5;
        u32x2* planes = (u32x2*)smem;
        uint16_t* bases = (uint16_t*)(planes + (size_t)NB * W);
        int bad = 0;
        if (lut_vec && (L & 31) == 0 && logW >= 4) {
            // Stage, coalesced and bank-conflict free: a wave packs 16
            // consecutive LDS positions of one level block. Lane 4g+q loads
            // the q-th 16-byte quarter (8 entries) of the block's row for
            // position p0+g; the four quarters' steps are merged by lane
            // shuffles and lane 4g writes the block's words.
            const int wl = tid & 63, wv = tid >> 6, nwv = nt >> 6;
            const int g = wl >> 2, q = wl & 3;
            const int logpg = logW - 4;
            const int units = NB << logpg;
            // Rounds of SU units per wave: all SU loads are issued before the
            // first unit is packed, so staging is not one load latency per unit.
            constexpr int SU = 8;
            for (int u0 = wv; u0 < units; u0 += nwv * SU) {
                u32x4 qv[SU];
#pragma unroll
                for (int s = 0; s < SU; ++s) {
                    const int u = u0 + s * nwv;
                    const int p = ((u & ((1 << logpg) - 1)) << 4) + g;
                    const int jj = ((p & ((1 << logq) - 1)) << LOGVEC) + (p >> logq);
                    qv[s] = u32x4{0u, 0u, 0u, 0u};
                    if (u < units && jj < weff) {
                        qv[s] = *(const u32x4*)(strip_lut + (size_t)jj * Lz +
                                                (size_t)(u >> logpg) * 32 + q * 8);
                    }
                }
#pragma unroll
                for (int s = 0; s < SU; ++s) {
                    const int u = u0 + s * nwv;
                    if (u >= units) break;  // uniform across the wave
                    const int blk = u >> logpg;
                    const int p = ((u & ((1 << logpg) - 1)) << 4) + g;
                    const int jj = ((p & ((1 << logq) - 1)) << LOGVEC) + (p >> logq);
                    const bool valid = jj < weff;
                    const u32x4 v4 = qv[s];
                    const uint32_t e[8] = {v4.x & 0xffffu, v4.x >> 16, v4.y & 0xffffu,
                                           v4.y >> 16,     v4.z & 0xffffu, v4.z >> 16,
                                           v4.w & 0xffffu, v4.w >> 16};
                    const uint32_t nxt = (uint32_t)__shfl_down((int)e[0], 1, 64);
                    uint32_t lo8 = 0, hi8 = 0, over = 0;
#pragma unroll
                    for (int i = 0; i < 8; ++i) {
                        // Step from entry 8q+i to 8q+i+1; block step 31 does not exist.
                        const uint32_t step =
                            i < 7 ? e[i + 1] - e[i] : (q < 3 ? nxt - e[7] : 0u);
                        over |= step > 3u;
                        lo8 |= (step & 1u) << i;
                        hi8 |= ((step >> 1) & 1u) << i;
                    }
                    uint32_t lo = lo8 << (q * 8), hi = hi8 << (q * 8);
                    lo |= (uint32_t)__shfl_xor((int)lo, 1, 64);
                    hi |= (uint32_t)__shfl_xor((int)hi, 1, 64);
                    lo |= (uint32_t)__shfl_xor((int)lo, 2, 64);
                    hi |= (uint32_t)__shfl_xor((int)hi, 2, 64);
                    if (valid) {
                        bad |= (int)over;
                        if (q == 0) {
                            u32x2 pl;
                            pl.x = lo;
                            pl.y = hi;
                            planes[blk * W + p] = pl;
                            bases[blk * W + p] = (uint16_t)e[0];
                        }
                    }
                }
            }
        } else {
            // Stage, general shapes: item = (detector jj, block), blocks fastest.
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
        }
        bad = packed_any(bad, planes);
        if (streams) {
            if (!bad) {
                stream_lines<VEC, UNROLL, NT>(
                    rin, rout, vo, line_stride, passes, [&](int k, uint32_t d) {
                        return g_packed(planes, bases, d, top, logW, (k << logq) + lane);
                    }, pass_adv);
            } else {
                const uint16_t* lrow = strip_lut + (size_t)j * Lz;
                stream_lines<VEC, UNROLL, NT>(
                    rin, rout, vo, line_stride, passes,
                    [&](int k, uint32_t d) { return g_glb(lrow + (size_t)k * Lz, d, top); }, pass_adv);
            }
        }
        __syncthreads();  // the tile may be restaged next
    }
}


// ---- fused LUT build + correction (batched requests) ------------------------------------

// Writes entries [v0, v0 + n) of one LUT row (n <= 8, values in e) to global
// memory: one 16-byte non-temporal store when the 8 entries are aligned (the
// tile reads its LUT from LDS, not back from memory), else 16-bit stores.
__device__ __forceinline__ void store_lut8(uint16_t* dst, const uint32_t* e, int n, bool vec16) {
    if (vec16 && n == 8) {
        u32x4 q;
        q.x = e[0] | (e[1] << 16);
        q.y = e[2] | (e[3] << 16);
        q.z = e[4] | (e[5] << 16);
        q.w = e[6] | (e[7] << 16);
        __builtin_nontemporal_store(q, (u32x4*)dst);
    } else {
        for (int k = 0; k < n; ++k) dst[k] = (uint16_t)e[k];
    }
}

// One LUT row encoded in the dense form by one wave: block blk's plane and
// header go to planes[blk * stride] and heads[blk * stride] (the
// [band][block][detector] layout of a dense workspace); a block the form
// cannot hold gets the header kDenseBad. src.fetch(v0, n) gives the n <= 8
// entries from level v0 packed two per word (evaluated from coefficients,
// or read from a LUT row); with dst they are also written there (L entries). 8 blocks per
// pass: lane 8g + q takes levels 64 (8 r + g) + 8q .. + 7, so a pass reads
// or stores 1 KiB of the row contiguously; the 8 lanes of a block decide its
// form (the cases of dense_encode) with xor-shuffles inside their group and
// OR their step bits together. Every lane of the wave must call it.
// Computes the LUT rows of band b, detectors [d0, d0 + weff) from their
// calibration coefficients straight into the LDS tile (raw or packed layout,
// as the correction tile reads them) and, if `write_lut`, also into the
// global LUT. Returns nonzero (the same on every thread) when a packed row
// has a step outside 0..3; the LDS tile is then unusable.
template <int VEC, int MODE>
__device__ __forceinline__ int build_strip(const double* __restrict__ coeffs, uint16_t* lut, int D,
                                           int L, int logW, int b, int d0, int weff,
                                           bool write_lut, bool lut_vec, void* smem) {
    constexpr int LOGVEC = log_vec<VEC>();
    const int W = 1 << logW;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int logq = logW - LOGVEC;
    const double lim = (double)L;
    const size_t row0 = (size_t)b * (size_t)D + (size_t)d0;
    int bad = 0;
    if constexpr (MODE == kRaw) {
        // Item = (detector j fastest, 8-level chunk): consecutive lanes write
        // consecutive LDS entries.
        uint16_t* tile = (uint16_t*)smem;
        const int chunks = (L + 7) >> 3;
        const int items = chunks << logW;
        for (int it = tid; it < items; it += nt) {
            const int j = it & (W - 1);
            const int c = it >> logW;
            if (j >= weff) continue;
            const double* a = coeffs + (row0 + (size_t)j) * 4;
            const double a0 = a[0], a1 = a[1], a2 = a[2], a3 = a[3];
            const int v0 = c * 8;
            const int n = min(8, L - v0);
            uint32_t e[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                e[k] = k < n ? lut_entry(a0, a1, a2, a3, v0 + k, lim) : 0u;
                if (k < n) tile[((v0 + k) << logW) + j] = (uint16_t)e[k];
            }
            if (write_lut) store_lut8(lut + (row0 + (size_t)j) * (size_t)L + v0, e, n, lut_vec);
        }
        __syncthreads();
    } else {
        // A wave evaluates one detector row at a time, 16 blocks of 32 levels
        // per pass: lane 4g + q computes levels 32 (16 r + g) + 8q .. + 7, so
        // the wave's global LUT stores cover 1 KiB of the row contiguously.
        // The four lanes of a block merge their step bits by lane shuffles.
        const int NB = (L + 31) >> 5;
        u32x2* planes = (u32x2*)smem;
        uint16_t* bases = (uint16_t*)(planes + (size_t)NB * W);
        const int lane = tid & 63;
        const int g = lane >> 2, q = lane & 3;
        const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
        const int nwv = nt >> 6;
        const int rounds = (NB + 15) >> 4;
        uint32_t maxstep = 0;
        for (int j = wv; j < weff; j += nwv) {
            const double* a = coeffs + (row0 + (size_t)j) * 4;
            const double a0 = a[0], a1 = a[1], a2 = a[2], a3 = a[3];
            uint16_t* dst = lut + (row0 + (size_t)j) * (size_t)L;
            const int p = ((j & (VEC - 1)) << logq) + (j >> LOGVEC);
            for (int r = 0; r < rounds; ++r) {
                const int blk = (r << 4) + g;
                const int v0 = (blk << 5) + (q << 3);
                const int n = max(0, min(8, L - v0));
                uint32_t e[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) e[k] = k < n ? lut_entry(a0, a1, a2, a3, v0 + k, lim) : 0u;
                if (write_lut && n > 0) store_lut8(dst + v0, e, n, lut_vec);
                // Step i of a block (bit i of the planes) is entry i+1 minus
                // entry i; a step that leaves the block or the row is 0.
                const uint32_t nxt = (uint32_t)__shfl_down((int)e[0], 1, 64);
                uint32_t lo8 = 0, hi8 = 0;
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const bool has = k < 7 ? k + 1 < n : (q < 3 && n == 8 && v0 + 8 < L);
                    const uint32_t step = has ? (k < 7 ? e[k + 1] : nxt) - e[k] : 0u;
                    maxstep = max(maxstep, step);  // wraps high when negative
                    lo8 |= (step & 1u) << k;
                    hi8 |= ((step >> 1) & 1u) << k;
                }
                uint32_t lo = lo8 << (q << 3), hi = hi8 << (q << 3);
                lo |= (uint32_t)__shfl_xor((int)lo, 1, 64);
                hi |= (uint32_t)__shfl_xor((int)hi, 1, 64);
                lo |= (uint32_t)__shfl_xor((int)lo, 2, 64);
                hi |= (uint32_t)__shfl_xor((int)hi, 2, 64);
                if (q == 0 && blk < NB) {
                    u32x2 pl;
                    pl.x = lo;
                    pl.y = hi;
                    planes[blk * W + p] = pl;
                    bases[blk * W + p] = (uint16_t)e[0];
                }
            }
        }
        bad = packed_any(maxstep > 3u ? 1 : 0, planes);
    }
    return bad;
}

// Writes the strip's LUT rows to global memory (second pass of a packed
// strip that cannot be packed and whose tile did not write them already).
__device__ __forceinline__ void write_strip(const double* __restrict__ coeffs, uint16_t* lut, int D,
                                            int L, int b, int d0, int weff, bool lut_vec) {
    const double lim = (double)L;
    const size_t row0 = (size_t)b * (size_t)D + (size_t)d0;
    const int chunks = (L + 7) >> 3;
    const int items = chunks * weff;
    for (int it = threadIdx.x; it < items; it += blockDim.x) {
        const int j = it / chunks;
        const int v0 = (it - j * chunks) * 8;
        const int n = min(8, L - v0);
        const double* a = coeffs + (row0 + (size_t)j) * 4;
        uint32_t e[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) e[k] = k < n ? lut_entry(a[0], a[1], a[2], a[3], v0 + k, lim) : 0u;
        store_lut8(lut + (row0 + (size_t)j) * (size_t)L + v0, e, n, lut_vec);
    }
}

// Global LUT gather that reads through the L2 (sc0), for rows this
// workgroup has just written.
__device__ __forceinline__ uint32_t g_glb_l2(__amdgpu_buffer_rsrc_t r, uint32_t row_off,
                                             uint32_t dnv, uint32_t top) {
    const uint32_t v = dnv < top ? dnv : top;
    return (uint16_t)__builtin_amdgcn_raw_buffer_load_b16(r, (int)(row_off + v * 2u), 0, 1);
}

// One fused tile of a batched request: build the strip's LUT in LDS from the
// coefficients (writing it to the global LUT too when write_lut), then
// correct lines [n0, n1) exactly as apply_tile does.
template <int VEC, int UNROLL, int MODE>
__device__ __forceinline__ void fused_tile(const double* __restrict__ coeffs, const uint16_t* dn,
                                           uint16_t* lut, uint16_t* out, int64_t N, int D, int L,
                                           int logW, int b, int d0, int weff, int64_t n0,
                                           int64_t n1, bool write_lut, void* smem, bool lut_vec) {
    constexpr int LOGVEC = log_vec<VEC>();
    const int bad = build_strip<VEC, MODE>(coeffs, lut, D, L, logW, b, d0, weff, write_lut,
                                           lut_vec, smem);
    if (n1 > n0) {
        const int tid = threadIdx.x;
        const int logq = logW - LOGVEC;
        const int lane = tid & ((1 << logq) - 1);
        const int rpp = blockDim.x >> logq;
        const int j = lane * VEC;
        const uint32_t top = (uint32_t)(L - 1);
        const size_t tile0 = ((size_t)b * (size_t)N + (size_t)n0) * (size_t)D + (size_t)d0;
        const uint32_t span = (uint32_t)((((size_t)(n1 - n0) - 1) * (size_t)D + (size_t)weff) * 2);
        const __amdgpu_buffer_rsrc_t rin = make_rsrc(dn + tile0, span);
        const __amdgpu_buffer_rsrc_t rout = make_rsrc(out + tile0, span);
        const uint32_t vo = (uint32_t)(((size_t)(tid >> logq) * (size_t)D + (size_t)j) * 2);
        const uint32_t line_stride = (uint32_t)rpp * (uint32_t)D * 2u;
        const int passes = (int)((n1 - n0 + (int64_t)rpp * UNROLL - 1) / ((int64_t)rpp * UNROLL));
        if constexpr (MODE == kRaw) {
            const uint16_t* tile = (const uint16_t*)smem;
            if (j < weff) {
                stream_lines<VEC, UNROLL, 0>(
                    rin, rout, vo, line_stride, passes,
                    [&](int k, uint32_t d) { return g_raw(tile, d, top, logW, j + k); });
            }
        } else {
            const int NB = (L + 31) >> 5;
            const u32x2* planes = (const u32x2*)smem;
            const uint16_t* bases = (const uint16_t*)(planes + (size_t)NB * (1 << logW));
            if (!bad) {
                if (j < weff) {
                    stream_lines<VEC, UNROLL, 0>(
                        rin, rout, vo, line_stride, passes, [&](int k, uint32_t d) {
                            return g_packed(planes, bases, d, top, logW, (k << logq) + lane);
                        });
                }
            } else {
                if (!write_lut) write_strip(coeffs, lut, D, L, b, d0, weff, lut_vec);
                __threadfence();
                __syncthreads();
                const size_t row0 = (size_t)b * (size_t)D + (size_t)d0;
                const __amdgpu_buffer_rsrc_t rl =
                    make_rsrc(lut + row0 * (size_t)L, (uint32_t)((size_t)weff * L * 2));
                if (j < weff) {
                    stream_lines<VEC, UNROLL, 0>(
                        rin, rout, vo, line_stride, passes, [&](int k, uint32_t d) {
                            return g_glb_l2(rl, (uint32_t)((j + k) * L * 2), d, top);
                        });
                }
            }
        }
    }
    __syncthreads();  // the tile may be rebuilt next
}

}  // namespace rc
