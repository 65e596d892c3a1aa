// Gradient-based Bayer demosaicing of RGGB mosaics, the second interpolation
// method the paper lists for its demosaicing task (§II, §III.A). The paper
// names the method without giving its steps; the one implemented is Hamilton
// and Adams' adaptive colour plane interpolation (U.S. Patent 5,629,734):
//   stage 1, green at R and B pixels: horizontal and vertical estimates, each
//     the mean of the two green neighbours plus a quarter of the second
//     difference of the pixel's own colour; the estimate along the smaller
//     gradient (|green difference| + |second difference|) is taken, the mean of
//     both on a tie;
//   stage 2, red and blue: the neighbours' colour differences X - G' averaged
//     and added to G' (at G pixels from the row or column pair, at R and B
//     pixels from the diagonal pair with the smaller gradient, both on a tie).
// Integer arithmetic, halves rounded up (quotients are arithmetic shifts of
// numerators with half the divisor added), interpolated values clamped to
// [0, 65535], indices outside the image mirrored about the edge sample.
//
// Layout and mapping: raw [images][H][W] uint16, rgb [images][3][H][W]. As in
// the bilinear kernel a lane owns 4 consecutive columns (8-byte loads and
// three 8-byte non-temporal stores per row) and walks down a band of rows.
// Stage 1 reaches two rows and columns, stage 2 one more, so a lane keeps a
// window of five raw rows (r-1 .. r+3) and three green rows (r-1 .. r+1) in
// registers: per output row r it unpacks raw row r+3 (loaded during the
// two previous rows), starts the load of row r+5, computes green row r+1 and
// finishes row r. The window is a ring of six slots, and the row loop is
// unrolled six times so the ring rotates by renaming, not by register moves,
// and the colour parity of every row is a compile-time constant.
// Neighbour columns come from the adjacent lanes by DPP wave shifts; the two
// lanes at a wave's edge load the 4 columns beyond it instead, and the wave
// computes the one green value beyond it that stage 2 needs (at column c0-1
// in B rows for lane 0, c0+4 in R rows for lane 63). On large launches the
// four waves of a workgroup hold adjacent columns and pass those values to
// each other through LDS instead, so only the workgroup's outer waves compute
// them. Virtual rows above and below the image are computed by the same code
// from mirrored raw rows: the stencils are symmetric, so they equal the
// mirrored green rows. Rows are read and written through buffer resources
// that span one image row, which makes idle lanes and loads beyond the image
// harmless (they read 0 and write nothing).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "device_ops.h"
#include "kernels.h"
#include "rc.h"
#include "runtime.h"

namespace rc {
namespace {

__device__ __forceinline__ int mirror_index(int i, int n) {
    return i < 0 ? -i : (i >= n ? 2 * (n - 1) - i : i);
}

// |a - b| + c on unsigned operands, one instruction.
__device__ __forceinline__ uint32_t sad(uint32_t a, uint32_t b, uint32_t c) {
    uint32_t r;
    asm("v_sad_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

__device__ __forceinline__ uint32_t absdiff(uint32_t a, uint32_t b) {
    uint32_t r;
    asm("v_sad_u32 %0, %1, %2, 0" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

// Lane i receives lane i-1's value (lane 0 keeps `old`), or lane i+1's (lane 63 keeps `old`).
__device__ __forceinline__ uint32_t from_lower_lane(uint32_t old, uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, 0x138, 0xf, 0xf, false);
}
__device__ __forceinline__ uint32_t from_upper_lane(uint32_t old, uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, 0x130, 0xf, 0xf, false);
}

// Per-lane constants of the column mapping. Rows are read and written through
// buffer resources that span exactly one image row, so accesses of idle lanes
// (c0 >= W) and of edge loads beyond the image read 0 and write nothing.
struct Lane {
    uint32_t off;       // byte offset of the lane's 4 samples in a row
    uint32_t edge_off;  // lane 0: off - 8, lane 63: off + 8, other lanes: out of range
    uint32_t ex_shift;  // where column c0-3 (lane 0) or c0+6 (lane 63) sits in the edge dword
    bool at_start;      // c0 == 0: columns -1, -2 are mirrored
    bool at_end;        // c0 + 4 == W: columns W, W+1 are mirrored
    int w;              // wave in the workgroup
    bool xl, xr;        // left / right neighbour wave in the workgroup (same band)
    uint32_t* xch;      // LDS exchange slots [row parity][wave]
};

// One raw row as a lane sees it: its 4 samples and the neighbour columns.
struct Raw {
    uint32_t v[4];    // columns c0 .. c0+3
    uint32_t l1, l2;  // columns c0-1, c0-2
    uint32_t r1, r2;  // columns c0+4, c0+5
    uint32_t exw;     // edge lanes: column c0-3 (lane 0) or c0+6 (lane 63) in bits ex_shift..+15
};

// One green row: the lane's 4 values and the two neighbour columns.
struct Green {
    uint32_t g[4];
    uint32_t gl, gr;  // columns c0-1 and c0+4
};

struct Load {
    uint2 q;     // the lane's 4 samples
    uint2 edge;  // lane 0: columns c0-4 .. c0-1; lane 63: columns c0+4 .. c0+7
};

__device__ __forceinline__ Load load_row(const uint16_t* row, uint32_t row_bytes, const Lane& ln) {
    const __amdgpu_buffer_rsrc_t r = make_rsrc(row, row_bytes);
    Load x;
    const u32x2 q = (u32x2)__builtin_amdgcn_raw_buffer_load_b64(r, (int)ln.off, 0, 0);
    const u32x2 e = (u32x2)__builtin_amdgcn_raw_buffer_load_b64(r, (int)ln.edge_off, 0, 0);
    x.q = make_uint2(q.x, q.y);
    x.edge = make_uint2(e.x, e.y);
    return x;
}

// EDGE: the wave holds column 0 or column W-1, so mirrored columns may be needed.
template <bool EDGE>
__device__ __forceinline__ Raw unpack(const Load& x, const Lane& ln) {
    Raw r;
    r.v[0] = x.q.x & 0xffffu;
    r.v[1] = x.q.x >> 16;
    r.v[2] = x.q.y & 0xffffu;
    r.v[3] = x.q.y >> 16;
    // Columns c0-2 | c0-1 << 16 and c0+4 | c0+5 << 16: from the adjacent
    // lanes, the edge load at the wave's edges, mirrored (2 | 1 << 16 and
    // W-2 | W-3 << 16, both the lane's own v2 | v1 << 16) at the image's.
    uint32_t left = from_lower_lane(x.edge.y, x.q.y);
    uint32_t right = from_upper_lane(x.edge.x, x.q.x);
    if (EDGE) {
        const uint32_t mir = (x.q.y & 0xffffu) | (x.q.x & 0xffff0000u);
        left = ln.at_start ? mir : left;
        right = ln.at_end ? mir : right;
    }
    r.l2 = left & 0xffffu;
    r.l1 = left >> 16;
    r.r1 = right & 0xffffu;
    r.r2 = right >> 16;
    r.exw = __builtin_amdgcn_alignbit(x.edge.y, x.edge.x, 16);  // c0-3 | c0-2 (lane 0), c0+5 | c0+6 (lane 63)
    return r;
}

__device__ __forceinline__ uint32_t ex_of(const Raw& r, const Lane& ln) {
    return (r.exw >> ln.ex_shift) & 0xffffu;
}

// Column t (-1 .. 4, relative to c0) of a raw row.
__device__ __forceinline__ uint32_t rat(const Raw& r, int t) {
    return t < 0 ? r.l1 : (t > 3 ? r.r1 : r.v[t]);
}

__device__ __forceinline__ uint32_t gat(const Green& g, int t) {
    return t < 0 ? g.gl : (t > 3 ? g.gr : g.g[t]);
}

__device__ __forceinline__ uint32_t clamp16(int v) { return (uint32_t)min(max(v, 0), 65535); }

// One of three estimates: e1 where g1 < g2, e2 where g2 < g1, their mean on a
// tie; e1 and e2 are numerators over 2^s. Each rounds half up to
// (2 e + 2^s) >> (s + 1), the tie to (e1 + e2 + 2^s) >> (s + 1): select
// first, round once.
template <int s>
__device__ __forceinline__ uint32_t pick(uint32_t g1, uint32_t g2, int e1, int e2) {
    const int one = g1 < g2 ? e1 : e2;
    const int n = g1 == g2 ? e1 + e2 : 2 * one;
    return clamp16((n + (1 << s)) >> (s + 1));
}

// Stage 1 at one R or B pixel: own sample c, green neighbours gl/gr/gu/gd,
// same-colour samples two away cl/cr/cu/cd.
__device__ __forceinline__ uint32_t green_at(uint32_t c, uint32_t gl, uint32_t gr, uint32_t gu,
                                             uint32_t gd, uint32_t cl, uint32_t cr, uint32_t cu,
                                             uint32_t cd) {
    const uint32_t c2 = 2 * c;
    const uint32_t sh = cl + cr, sv = cu + cd;
    const uint32_t dh = sad(gl, gr, absdiff(c2, sh));  // |Gl - Gr| + |2C - Cl - Cr|
    const uint32_t dv = sad(gu, gd, absdiff(c2, sv));
    const int eh = (int)(2 * (gl + gr + c)) - (int)sh;  // 2 (Gl + Gr) + 2C - Cl - Cr
    const int ev = (int)(2 * (gu + gd + c)) - (int)sv;
    return pick<2>(dh, dv, eh, ev);
}

// Green row from raw rows two above (u2) to two below (d2), with its neighbour
// columns: from the adjacent lanes, mirrored at the image edges, or computed
// by the wave's edge lanes. odd: a B row, non-green at odd columns (a
// constant once the row loop is unrolled).
template <bool EDGE, bool XCH>
__device__ __forceinline__ Green green_row(bool odd, const Raw& u2, const Raw& u1, const Raw& m,
                                           const Raw& d1, const Raw& d2, const Lane& ln) {
    Green G;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        if (((j & 1) != 0) == odd) {
            G.g[j] = green_at(m.v[j], rat(m, j - 1), rat(m, j + 1), u1.v[j], d1.v[j],
                              j >= 2 ? m.v[j - 2] : (j == 1 ? m.l1 : m.l2),
                              j <= 1 ? m.v[j + 2] : (j == 2 ? m.r1 : m.r2), u2.v[j], d2.v[j]);
        } else {
            G.g[j] = m.v[j];
        }
    }
    // The green value just beyond the wave: column c0-1 (odd, so non-green in
    // B rows) for lane 0, column c0+4 (even, non-green in R rows) for lane 63.
    // Every lane evaluates it; only the edge lanes keep the result.
    // XCH: the four waves of the workgroup hold adjacent columns of one band,
    // so a wave publishes the value its neighbour needs (lane 63's g[3] for
    // B rows, lane 0's g[0] for R rows) in LDS, and only the waves at the
    // workgroup's edges compute theirs. One barrier per green row, the same
    // number in every wave (same band, no wave leaves early); a slot is
    // rewritten two rows later, after the next row's barrier.
    uint32_t extra;
    bool have = false;
    if (XCH) {
        const int lane = threadIdx.x & 63;
        uint32_t* slot = ln.xch + (odd ? 0 : 4);
        if (odd) {
            if (lane == 63) slot[ln.w] = G.g[3];
        } else {
            if (lane == 0) slot[ln.w] = G.g[0];
        }
        __syncthreads();
        have = odd ? ln.xl : ln.xr;
        if (have) extra = slot[odd ? ln.w - 1 : ln.w + 1];
    }
    if (!have) {
        const uint32_t ex = ex_of(m, ln);
        extra = odd ? green_at(m.l1, m.l2, m.v[0], u1.l1, d1.l1, ex, m.v[1], u2.l1, d2.l1)
                    : green_at(m.r1, m.v[3], m.r2, u1.r1, d1.r1, m.v[2], ex, u2.r1, d2.r1);
    }
    G.gl = from_lower_lane(odd ? extra : m.l1, G.g[3]);
    G.gr = from_upper_lane(odd ? m.r1 : extra, G.g[0]);
    if (EDGE) {
        G.gl = ln.at_start ? G.g[1] : G.gl;  // column -1 reads 1
        G.gr = ln.at_end ? G.g[2] : G.gr;    // column W reads W-2
    }
    return G;
}

// Stage 2 at a G pixel with green g0: a missing colour from the pair x1, x2
// with greens g1, g2.
__device__ __forceinline__ uint32_t pair_at(uint32_t x1, uint32_t x2, uint32_t g1, uint32_t g2,
                                            uint32_t g0x2p1) {
    return clamp16((int)(x1 + x2 + g0x2p1 - (g1 + g2)) >> 1);
}

// Stage 2 at an R or B pixel j with green g0: the other of R and B from the
// diagonal pair with the smaller gradient.
__device__ __forceinline__ uint32_t diag_at(const Raw& u, const Raw& d, const Green& gu,
                                            const Green& gd, int j, uint32_t g0) {
    const uint32_t n1 = rat(u, j - 1), n2 = rat(d, j + 1);
    const uint32_t p1 = rat(u, j + 1), p2 = rat(d, j - 1);
    const uint32_t g2 = 2 * g0;
    const uint32_t gn = gat(gu, j - 1) + gat(gd, j + 1);
    const uint32_t gp = gat(gu, j + 1) + gat(gd, j - 1);
    const uint32_t dn = sad(n1, n2, absdiff(g2, gn));
    const uint32_t dp = sad(p1, p2, absdiff(g2, gp));
    const int sn = (int)(n1 + n2 + g2) - (int)gn;
    const int sp = (int)(p1 + p2 + g2) - (int)gp;
    return pick<1>(dn, dp, sn, sp);
}

__device__ __forceinline__ void store_nt(__amdgpu_buffer_rsrc_t r, uint32_t off, const uint32_t* v) {
    i32x2 w;
    w.x = (int)(v[0] | (v[1] << 16));
    w.y = (int)(v[2] | (v[3] << 16));
    // Non-temporal: the planes are written once and not read back here.
    __builtin_amdgcn_raw_buffer_store_b64(w, r, (int)off, 0, 2);
}

// Output row r from raw rows r-1, r, r+1 and green rows r-1, r, r+1; `row`
// is row r of the R plane, the G and B planes follow at `plane` samples.
__device__ __forceinline__ void finish_row(bool red_row, const Raw& u, const Raw& m, const Raw& d,
                                           const Green& gu, const Green& gm, const Green& gd,
                                           uint16_t* row, size_t plane, uint32_t row_bytes,
                                           const Lane& ln) {
    uint32_t R[4], B[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t g0 = gm.g[j];
        const bool even = (j & 1) == 0;  // c0 is a multiple of 4
        if (red_row == even) {           // R pixel (red row) or B pixel (blue row)
            const uint32_t other = diag_at(u, d, gu, gd, j, g0);
            R[j] = red_row ? m.v[j] : other;
            B[j] = red_row ? other : m.v[j];
        } else {                         // G pixel
            const uint32_t g0x2p1 = 2 * g0 + 1;
            const uint32_t hor = pair_at(rat(m, j - 1), rat(m, j + 1), gat(gm, j - 1),
                                         gat(gm, j + 1), g0x2p1);
            const uint32_t ver = pair_at(u.v[j], d.v[j], gu.g[j], gd.g[j], g0x2p1);
            R[j] = red_row ? hor : ver;
            B[j] = red_row ? ver : hor;
        }
    }
    store_nt(make_rsrc(row, row_bytes), ln.off, R);
    store_nt(make_rsrc(row + plane, row_bytes), ln.off, gm.g);
    store_nt(make_rsrc(row + 2 * plane, row_bytes), ln.off, B);
}

// One band of rows [r0, r1) of one image, for the wave's 256 columns.
template <bool EDGE, bool XCH>
__device__ __forceinline__ void run_band(const uint16_t* im, uint16_t* out, int H, int W, int r0,
                                         int r1, const Lane& ln) {
    const size_t plane = (size_t)H * (size_t)W;
    const uint32_t row_bytes = (uint32_t)W * 2u;
    auto row_of = [&](int rr) { return im + (size_t)mirror_index(rr, H) * (size_t)W; };
    auto fetch = [&](int rr) { return load_row(row_of(rr), row_bytes, ln); };

    // Ring slot of raw row x and green row x: (x - r0 + 1) mod 6. Six slots
    // (five in use) and a six-fold unrolled loop: r0 and the loop step are
    // even, so every row's colour parity is known at compile time.
    Raw U[6];
    Green G[6];
    {
        const Raw a = unpack<EDGE>(fetch(r0 - 3), ln);
        const Raw b = unpack<EDGE>(fetch(r0 - 2), ln);
        U[0] = unpack<EDGE>(fetch(r0 - 1), ln);
        U[1] = unpack<EDGE>(fetch(r0), ln);
        U[2] = unpack<EDGE>(fetch(r0 + 1), ln);
        U[3] = unpack<EDGE>(fetch(r0 + 2), ln);
        G[0] = green_row<EDGE, XCH>(true, a, b, U[0], U[1], U[2], ln);
        G[1] = green_row<EDGE, XCH>(false, b, U[0], U[1], U[2], U[3], ln);
    }
    // Two rows in flight: L[1] holds the odd rows after r0 + 2, L[0] the even.
    Load L[2];
    L[1] = fetch(r0 + 3);
    L[0] = fetch(r0 + 4);
    for (int base = r0; base < r1; base += 6) {
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const int r = base + k;
            if (r >= r1) break;
            // Raw row r+3 arrives; row r+5 is loaded while this row and the
            // next are computed (rows beyond r1 + 2 are never needed).
            U[(k + 4) % 6] = unpack<EDGE>(L[(k + 1) % 2], ln);
            if (r + 3 <= r1) L[(k + 1) % 2] = fetch(r + 5);
            const bool even = (k & 1) == 0;  // row r is an R row
            G[(k + 2) % 6] = green_row<EDGE, XCH>(even, U[k], U[(k + 1) % 6], U[(k + 2) % 6],
                                             U[(k + 3) % 6], U[(k + 4) % 6], ln);
            finish_row(even, U[k], U[(k + 1) % 6], U[(k + 2) % 6], G[k], G[(k + 1) % 6],
                       G[(k + 2) % 6], out + (size_t)r * (size_t)W, plane, row_bytes, ln);
        }
    }
}

__global__ __launch_bounds__(256) void k_demosaic_gradient(const uint16_t* __restrict__ raw,
                                                           uint16_t* __restrict__ rgb,
                                                           int32_t images, int32_t H, int32_t W,
                                                           int32_t band, int32_t bands,
                                                           int32_t col_waves, int32_t exchange) {
    const int lane = threadIdx.x & 63;
    // Wave-uniform (scalar) from here: the wave index and everything derived from it.
    __shared__ uint32_t xch[8];
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int wave = __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x >> 6)) + wv;
    const int per_image = bands * col_waves;
    if (wave >= images * per_image) return;  // whole waves of the last block
    const int img = wave / per_image;
    const int rem = wave - img * per_image;
    const int bi = rem / col_waves;
    const int cw = rem - bi * col_waves;
    const int c0 = (cw * 64 + lane) * 4;
    Lane ln;
    ln.off = (uint32_t)c0 * 2u;
    ln.edge_off = lane == 0 ? ln.off - 8u : (lane == 63 ? ln.off + 8u : 0xfffffff0u);
    ln.ex_shift = lane == 0 ? 0u : 16u;
    ln.at_start = c0 == 0;
    ln.at_end = c0 + 4 == W;
    ln.w = wv;
    ln.xl = wv > 0;
    ln.xr = wv < 3;
    ln.xch = xch;
    const int r0 = bi * band;
    const int r1 = min(H, r0 + band);
    const size_t plane = (size_t)H * (size_t)W;
    const uint16_t* im = raw + (size_t)img * plane;
    uint16_t* out = rgb + (size_t)img * 3 * plane;
    if (exchange) {
        if (cw == 0 || cw == col_waves - 1)
            run_band<true, true>(im, out, H, W, r0, r1, ln);
        else
            run_band<false, true>(im, out, H, W, r0, r1, ln);
    } else {
        if (cw == 0 || cw == col_waves - 1)
            run_band<true, false>(im, out, H, W, r0, r1, ln);
        else
            run_band<false, false>(im, out, H, W, r0, r1, ln);
    }
}

}  // namespace

hipError_t launch_demosaic_gradient(const uint16_t* raw, int32_t images, int32_t H, int32_t W,
                                    uint16_t* rgb, int cus, hipStream_t stream) {
    cus = cus > 0 ? cus : 256;
    const int col_waves = (W / 4 + 63) / 64;
    // Bands of about 16 waves per CU over the launch and at least 8 rows (each
    // band re-reads 5 halo rows and recomputes 2 green rows; on one 2048 x 2048
    // image 8-row bands still beat 16-row ones, which leave one wave per SIMD).
    const int64_t target = (int64_t)16 * cus;
    const int64_t col_total = (int64_t)images * col_waves;
    int64_t band = ((int64_t)H * col_total + target - 1) / target;
    band = band < 8 ? 8 : (band > 128 ? 128 : band);
    band = (band + 1) & ~(int64_t)1;  // whole Bayer rows
    const int bands = (int)(((int64_t)H + band - 1) / band);
    const int64_t waves = col_total * bands;
    const int64_t blocks = (waves + 3) / 4;
    // The LDS exchange needs every workgroup inside one band (whole groups of
    // 4 column waves). Its barriers cost more than they save on launches of
    // up to 8 waves per CU (one 2048 x 2048 image in 8-row bands, 8 waves per
    // CU: 9.6 vs 9.0 us), and save about 4 % on large ones (16 images: 101 vs
    // 106 us).
    const int exchange = (col_waves % 4 == 0 && waves > 8 * (int64_t)cus) ? 1 : 0;
    hipLaunchKernelGGL(k_demosaic_gradient, dim3((unsigned)blocks), dim3(256), 0, stream, raw, rgb,
                       images, H, W, (int)band, bands, col_waves, exchange);
    return hipGetLastError();
}

}  // namespace rc

using namespace rc;

extern "C" {

rc_status rc_demosaic_gradient(const uint16_t* raw, int32_t images, int32_t height,
                               int32_t width, uint16_t* rgb, hipStream_t stream) {
    if (images < 0 || height < 0 || width < 0) return RC_EINVAL;
    int64_t px = 0, n = 0;
    if (!mul_ok(height, width, &px) || !mul_ok(px, images, &n) || n > INT64_MAX / 8)
        return RC_EINVAL;
    if (n == 0) return RC_OK;
    if (height % 2 || width % 4 || height < 4 || width < 4) return RC_EINVAL;
    if (!raw || !rgb) return RC_EINVAL;
    if (((uintptr_t)raw | (uintptr_t)rgb) & 7u) return RC_EINVAL;
    if (overlaps(raw, (size_t)n * 2, rgb, (size_t)n * 6)) return RC_EINVAL;
    // Wave indices are 32-bit: images x bands x column waves < 2^31 (bands of >= 8 rows).
    if ((int64_t)images * (height / 8 + 1) * ((width / 4 + 63) / 64) >= ((int64_t)1 << 31))
        return RC_EINVAL;
    const DeviceInfo* di = current_device();
    if (!di) return RC_EHIP;
    hipError_t e = launch_demosaic_gradient(raw, images, height, width, rgb, di->cus, stream);
    return e == hipSuccess ? RC_OK : hip_fail(e);
}

}  // extern "C"
