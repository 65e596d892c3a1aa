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
// previous row), starts the load of row r+4, computes green row r+1 and
// finishes row r. The window is a ring of five slots, and the row loop is
// unrolled five times so the ring rotates by renaming, not by register moves.
// Neighbour columns come from the adjacent lanes by lane shuffles; the two
// lanes at a wave's edge load the 4 columns beyond it instead, and compute the
// one green value beyond the wave that stage 2 needs (at column c0-1 in B
// rows for lane 0, c0+4 in R rows for lane 63). Virtual rows above and below
// the image are computed by the same code from mirrored raw rows: the
// stencils are symmetric, so they equal the mirrored green rows. No LDS.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"
#include "rc.h"
#include "runtime.h"

namespace rc {
namespace {

__device__ __forceinline__ int mirror_index(int i, int n) {
    return i < 0 ? -i : (i >= n ? 2 * (n - 1) - i : i);
}

// One raw row as a lane sees it: its 4 samples and the neighbour columns.
struct Raw {
    int v[4];    // columns c0 .. c0+3
    int l1, l2;  // columns c0-1, c0-2
    int r1, r2;  // columns c0+4, c0+5
    int ex;      // column c0-3 (lane 0) or c0+6 (lane 63), for the green beyond the wave
};

// One green row: the lane's 4 values and the two neighbour columns.
struct Green {
    int g[4];
    int gl, gr;  // columns c0-1 and c0+4
};

struct Load {
    uint2 q;     // the lane's 4 samples
    uint2 edge;  // lane 0: columns c0-4 .. c0-1; lane 63: columns c0+4 .. c0+7
};

__device__ __forceinline__ Load load_row(const uint16_t* im, int W, int r, int c0, bool valid,
                                         int lane) {
    Load x;
    x.q = make_uint2(0u, 0u);
    x.edge = make_uint2(0u, 0u);
    if (valid) {
        const uint16_t* p = im + (size_t)r * (size_t)W;
        x.q = *(const uint2*)(p + c0);
        if (lane == 0 && c0 > 0) x.edge = *(const uint2*)(p + c0 - 4);
        if (lane == 63 && c0 + 4 < W) x.edge = *(const uint2*)(p + c0 + 4);
    }
    return x;
}

__device__ __forceinline__ Raw unpack(const Load& x, int c0, int W, int lane) {
    Raw r;
    r.v[0] = (int)(x.q.x & 0xffffu);
    r.v[1] = (int)(x.q.x >> 16);
    r.v[2] = (int)(x.q.y & 0xffffu);
    r.v[3] = (int)(x.q.y >> 16);
    const uint32_t left = (uint32_t)__shfl_up((int)x.q.y, 1, 64);    // c0-2 | c0-1 << 16
    const uint32_t right = (uint32_t)__shfl_down((int)x.q.x, 1, 64); // c0+4 | c0+5 << 16
    if (c0 == 0) {  // mirrored: -1 reads 1, -2 reads 2
        r.l1 = r.v[1];
        r.l2 = r.v[2];
    } else if (lane == 0) {
        r.l1 = (int)(x.edge.y >> 16);
        r.l2 = (int)(x.edge.y & 0xffffu);
    } else {
        r.l1 = (int)(left >> 16);
        r.l2 = (int)(left & 0xffffu);
    }
    if (c0 + 4 == W) {  // mirrored: W reads W-2, W+1 reads W-3
        r.r1 = r.v[2];
        r.r2 = r.v[1];
    } else if (lane == 63) {
        r.r1 = (int)(x.edge.x & 0xffffu);
        r.r2 = (int)(x.edge.x >> 16);
    } else {
        r.r1 = (int)(right & 0xffffu);
        r.r2 = (int)(right >> 16);
    }
    // Only lane 0 (c0 > 0) and lane 63 (c0 + 4 < W) use it.
    r.ex = lane == 0 ? (int)(x.edge.x >> 16) : (int)(x.edge.y & 0xffffu);
    return r;
}

// Column t (-1 .. 4, relative to c0) of a raw row.
__device__ __forceinline__ int rat(const Raw& r, int t) {
    return t < 0 ? r.l1 : (t > 3 ? r.r1 : r.v[t]);
}

__device__ __forceinline__ int gat(const Green& g, int t) {
    return t < 0 ? g.gl : (t > 3 ? g.gr : g.g[t]);
}

__device__ __forceinline__ int clamp16(int v) { return min(max(v, 0), 65535); }

// Stage 1 at one R or B pixel: own sample c, green neighbours gl/gr/gu/gd,
// same-colour samples two away cl/cr/cu/cd.
__device__ __forceinline__ int green_at(int c, int gl, int gr, int gu, int gd, int cl, int cr,
                                        int cu, int cd) {
    const int lh = 2 * c - cl - cr;
    const int lv = 2 * c - cu - cd;
    const int dh = abs(gl - gr) + abs(lh);
    const int dv = abs(gu - gd) + abs(lv);
    const int eh = 2 * (gl + gr) + lh;
    const int ev = 2 * (gu + gd) + lv;
    const int g = dh < dv ? (eh + 2) >> 2 : (dv < dh ? (ev + 2) >> 2 : (eh + ev + 4) >> 3);
    return clamp16(g);
}

// Green row rr from raw rows rr-2 .. rr+2 (u2 .. d2), with its neighbour
// columns: from the adjacent lanes, mirrored at the image edges, or computed
// by the wave's edge lanes.
__device__ __forceinline__ Green green_row(int rr, const Raw& u2, const Raw& u1, const Raw& m,
                                           const Raw& d1, const Raw& d2, int c0, int W,
                                           int lane) {
    Green G;
    const bool odd = (rr & 1) != 0;  // B row: non-green at odd columns
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
    const int extra = odd ? green_at(m.l1, m.l2, m.v[0], u1.l1, d1.l1, m.ex, m.v[1], u2.l1, d2.l1)
                          : green_at(m.r1, m.v[3], m.r2, u1.r1, d1.r1, m.v[2], m.ex, u2.r1, d2.r1);
    const int from_left = __shfl_up(G.g[3], 1, 64);
    const int from_right = __shfl_down(G.g[0], 1, 64);
    if (c0 == 0) G.gl = G.g[1];
    else if (lane == 0) G.gl = odd ? extra : m.l1;
    else G.gl = from_left;
    if (c0 + 4 == W) G.gr = G.g[2];
    else if (lane == 63) G.gr = odd ? m.r1 : extra;
    else G.gr = from_right;
    return G;
}

// Stage 2 at one pixel: a missing colour from a pair of samples x1, x2 with
// greens g1, g2, at a pixel with green g0.
__device__ __forceinline__ int pair_at(int x1, int x2, int g1, int g2, int g0) {
    return clamp16((x1 + x2 + 2 * g0 - g1 - g2 + 1) >> 1);
}

__device__ __forceinline__ int diag_at(const Raw& u, const Raw& d, const Green& gu,
                                       const Green& gd, int j, int g0) {
    const int n1 = rat(u, j - 1), n2 = rat(d, j + 1);
    const int p1 = rat(u, j + 1), p2 = rat(d, j - 1);
    const int ln = 2 * g0 - gat(gu, j - 1) - gat(gd, j + 1);
    const int lp = 2 * g0 - gat(gu, j + 1) - gat(gd, j - 1);
    const int dn = abs(n1 - n2) + abs(ln);
    const int dp = abs(p1 - p2) + abs(lp);
    const int sn = n1 + n2 + ln, sp = p1 + p2 + lp;
    const int v = dn < dp ? (sn + 1) >> 1 : (dp < dn ? (sp + 1) >> 1 : (sn + sp + 2) >> 2);
    return clamp16(v);
}

__device__ __forceinline__ void store_pair(uint16_t* p, const int* v) {
    uint32_t* q = (uint32_t*)p;
    __builtin_nontemporal_store((uint32_t)v[0] | ((uint32_t)v[1] << 16), q);
    __builtin_nontemporal_store((uint32_t)v[2] | ((uint32_t)v[3] << 16), q + 1);
}

// Output row r from raw rows r-1, r, r+1 and green rows r-1, r, r+1.
__device__ __forceinline__ void finish_row(int r, const Raw& u, const Raw& m, const Raw& d,
                                           const Green& gu, const Green& gm, const Green& gd,
                                           uint16_t* out, size_t plane, int W, int c0,
                                           bool valid) {
    int R[4], B[4];
    const bool red_row = (r & 1) == 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int g0 = gm.g[j];
        const bool even = (j & 1) == 0;  // c0 is a multiple of 4
        if (red_row == even) {           // R pixel (red row) or B pixel (blue row)
            const int other = diag_at(u, d, gu, gd, j, g0);
            R[j] = red_row ? m.v[j] : other;
            B[j] = red_row ? other : m.v[j];
        } else {                         // G pixel
            const int hor = pair_at(rat(m, j - 1), rat(m, j + 1), gat(gm, j - 1), gat(gm, j + 1), g0);
            const int ver = pair_at(u.v[j], d.v[j], gu.g[j], gd.g[j], g0);
            R[j] = red_row ? hor : ver;
            B[j] = red_row ? ver : hor;
        }
    }
    if (valid) {
        const size_t o = (size_t)r * (size_t)W + (size_t)c0;
        // Non-temporal: the planes are written once and not read back here.
        store_pair(out + o, R);
        store_pair(out + plane + o, gm.g);
        store_pair(out + 2 * plane + o, B);
    }
}

__global__ __launch_bounds__(256) void k_demosaic_gradient(const uint16_t* __restrict__ raw,
                                                           uint16_t* __restrict__ rgb,
                                                           int32_t images, int32_t H, int32_t W,
                                                           int32_t band, int32_t bands,
                                                           int32_t col_waves) {
    const int lane = threadIdx.x & 63;
    const int wave = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int per_image = bands * col_waves;
    if (wave >= images * per_image) return;  // whole waves of the last block
    const int img = wave / per_image;
    const int rem = wave - img * per_image;
    const int bi = rem / col_waves;
    const int cw = rem - bi * col_waves;
    const int c0 = (cw * 64 + lane) * 4;
    const bool valid = c0 < W;
    const int r0 = bi * band;
    const int r1 = min(H, r0 + band);
    const size_t plane = (size_t)H * (size_t)W;
    const uint16_t* im = raw + (size_t)img * plane;
    uint16_t* out = rgb + (size_t)img * 3 * plane;

    auto fetch = [&](int rr) {
        return unpack(load_row(im, W, mirror_index(rr, H), c0, valid, lane), c0, W, lane);
    };
    // Ring slot of raw row x and green row x: (x - r0 + 1) mod 5.
    Raw U[5];
    Green G[5];
    {
        const Raw a = fetch(r0 - 3);
        const Raw b = fetch(r0 - 2);
        U[0] = fetch(r0 - 1);
        U[1] = fetch(r0);
        U[2] = fetch(r0 + 1);
        U[3] = fetch(r0 + 2);
        G[0] = green_row(r0 - 1, a, b, U[0], U[1], U[2], c0, W, lane);
        G[1] = green_row(r0, b, U[0], U[1], U[2], U[3], c0, W, lane);
    }
    Load next = load_row(im, W, mirror_index(r0 + 3, H), c0, valid, lane);
    for (int base = r0; base < r1; base += 5) {
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            const int r = base + k;
            if (r >= r1) break;
            // Raw row r+3 arrives; row r+4 is loaded while this row is computed
            // (rows beyond r1 + 2 are never needed).
            U[(k + 4) % 5] = unpack(next, c0, W, lane);
            next = load_row(im, W, mirror_index(r + 4, H), c0, valid && r + 2 <= r1, lane);
            G[(k + 2) % 5] = green_row(r + 1, U[k], U[(k + 1) % 5], U[(k + 2) % 5],
                                       U[(k + 3) % 5], U[(k + 4) % 5], c0, W, lane);
            finish_row(r, U[k], U[(k + 1) % 5], U[(k + 2) % 5], G[k], G[(k + 1) % 5],
                       G[(k + 2) % 5], out, plane, W, c0, valid);
        }
    }
}

}  // namespace

hipError_t launch_demosaic_gradient(const uint16_t* raw, int32_t images, int32_t H, int32_t W,
                                    uint16_t* rgb, int cus, hipStream_t stream) {
    const int col_waves = (W / 4 + 63) / 64;
    // Bands of about 16 waves per CU over the launch; at least 16 rows, since
    // each band re-reads 5 halo rows and recomputes 2 green rows.
    const int64_t target = (int64_t)16 * (cus > 0 ? cus : 256);
    const int64_t col_total = (int64_t)images * col_waves;
    int64_t band = ((int64_t)H * col_total + target - 1) / target;
    band = band < 16 ? 16 : (band > 128 ? 128 : band);
    band = (band + 1) & ~(int64_t)1;  // whole Bayer rows
    const int bands = (int)(((int64_t)H + band - 1) / band);
    const int64_t waves = col_total * bands;
    const int64_t blocks = (waves + 3) / 4;
    hipLaunchKernelGGL(k_demosaic_gradient, dim3((unsigned)blocks), dim3(256), 0, stream, raw, rgb,
                       images, H, W, (int)band, bands, col_waves);
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
    // Wave indices are 32-bit: images x bands x column waves < 2^31.
    if ((int64_t)images * (height / 16 + 1) * ((width / 4 + 63) / 64) >= ((int64_t)1 << 31))
        return RC_EINVAL;
    const DeviceInfo* di = current_device();
    if (!di) return RC_EHIP;
    hipError_t e = launch_demosaic_gradient(raw, images, height, width, rgb, di->cus, stream);
    return e == hipSuccess ? RC_OK : hip_fail(e);
}

}  // extern "C"
