// Bilinear Bayer demosaicing (§III.A, case study 1 of the paper) of RGGB
// mosaics: every pixel keeps its own sample; each missing colour is the
// average, rounded half up, of that colour's samples among the 8 direct
// neighbours (4 cross or 4 diagonal neighbours at red and blue pixels, the 2
// horizontal or 2 vertical ones at green pixels); indices outside the image
// are mirrored about the edge sample.
//
// Layout and mapping: raw [images][H][W] uint16, rgb [images][3][H][W]. A
// lane owns 4 consecutive columns (one 8-byte load per row, three 8-byte
// non-temporal stores per row, so a wave moves 512 contiguous bytes per
// instruction) and walks down a band of rows with a three-row window in
// registers: each row is loaded once (a band's two halo rows aside), two rows
// ahead of the one being computed. The ring of three rows rotates by
// renaming in a six-fold unrolled loop, so each row's colour parity is a
// compile-time constant. The left and right neighbour columns come from the
// adjacent lanes by DPP wave shifts; only the two lanes at a wave's edge load
// them. Rows go through buffer resources that span one image row, so idle
// lanes and loads beyond the image need no guards. No LDS.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "device_ops.h"
#include "kernels.h"
#include "rc.h"
#include "runtime.h"

namespace rc {
namespace {

__device__ __forceinline__ int mirror_row(int r, int H) {
    return r < 0 ? -r : (r >= H ? 2 * (H - 1) - r : r);
}

// Lane i receives lane i-1's value (lane 0 keeps `old`), or lane i+1's (lane 63 keeps `old`).
__device__ __forceinline__ uint32_t from_lower(uint32_t old, uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, 0x138, 0xf, 0xf, false);
}
__device__ __forceinline__ uint32_t from_upper(uint32_t old, uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, 0x130, 0xf, 0xf, false);
}

// Per-lane constants. Rows are read and written through buffer resources that
// span exactly one image row: loads of idle lanes (c0 >= W) and edge loads
// beyond the image read 0, stores of idle lanes write nothing.
struct Lane {
    uint32_t off;       // byte offset of the lane's 4 samples in a row
    uint32_t edge_off;  // lane 0: columns c0-2, c0-1; lane 63: c0+4, c0+5; others out of range
    bool at_start;      // c0 == 0: column -1 reads 1
    bool at_end;        // c0 + 4 == W: column W reads W-2
};

struct Load {
    u32x2 q;        // the lane's 4 samples
    uint32_t edge;  // the 2 samples beyond the wave (edge lanes)
};

struct Row {
    uint32_t v[4];  // columns c0 .. c0+3
    uint32_t w, e;  // columns c0-1 and c0+4
};

__device__ __forceinline__ Load load_row(const uint16_t* row, uint32_t row_bytes, const Lane& ln) {
    const __amdgpu_buffer_rsrc_t r = make_rsrc(row, row_bytes);
    Load x;
    x.q = (u32x2)__builtin_amdgcn_raw_buffer_load_b64(r, (int)ln.off, 0, 0);
    x.edge = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(r, (int)ln.edge_off, 0, 0);
    return x;
}

template <bool EDGE>
__device__ __forceinline__ Row unpack(const Load& x, const Lane& ln) {
    Row r;
    r.v[0] = x.q.x & 0xffffu;
    r.v[1] = x.q.x >> 16;
    r.v[2] = x.q.y & 0xffffu;
    r.v[3] = x.q.y >> 16;
    r.w = from_lower(x.edge, x.q.y) >> 16;      // column c0-1: the left lane's v3
    r.e = from_upper(x.edge, x.q.x) & 0xffffu;  // column c0+4: the right lane's v0
    if (EDGE) {
        r.w = ln.at_start ? r.v[1] : r.w;
        r.e = ln.at_end ? r.v[2] : r.e;
    }
    return r;
}

// Neighbour k of column j (0..3) in a row: k = -1 left, 0 self, +1 right.
__device__ __forceinline__ uint32_t at(const Row& r, int j, int k) {
    const int t = j + k;
    return t < 0 ? r.w : (t > 3 ? r.e : r.v[t]);
}

__device__ __forceinline__ void store_nt(__amdgpu_buffer_rsrc_t r, uint32_t off, const uint32_t* v) {
    i32x2 w;
    w.x = (int)(v[0] | (v[1] << 16));
    w.y = (int)(v[2] | (v[3] << 16));
    // Non-temporal: the planes are written once and not read back here.
    __builtin_amdgcn_raw_buffer_store_b64(w, r, (int)off, 0, 2);
}

// Output row r (an R row when red_row, a constant once the loop is unrolled)
// from rows r-1 (P), r (C) and r+1 (N); `row` is row r of the R plane.
__device__ __forceinline__ void finish_row(bool red_row, const Row& P, const Row& C, const Row& N,
                                           uint16_t* row, size_t plane, uint32_t row_bytes,
                                           const Lane& ln) {
    uint32_t R[4], G[4], B[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t own = C.v[j];
        const uint32_t hor = at(C, j, -1) + at(C, j, 1);
        const uint32_t ver = P.v[j] + N.v[j];
        if (red_row == ((j & 1) == 0)) {  // R pixel (R row) or B pixel (B row); c0 is even
            const uint32_t cross = (hor + ver + 2) >> 2;
            const uint32_t dg = (at(P, j, -1) + at(P, j, 1) + at(N, j, -1) + at(N, j, 1) + 2) >> 2;
            R[j] = red_row ? own : dg;
            G[j] = cross;
            B[j] = red_row ? dg : own;
        } else {                            // G pixel
            const uint32_t h2 = (hor + 1) >> 1, v2 = (ver + 1) >> 1;
            R[j] = red_row ? h2 : v2;
            G[j] = own;
            B[j] = red_row ? v2 : h2;
        }
    }
    store_nt(make_rsrc(row, row_bytes), ln.off, R);
    store_nt(make_rsrc(row + plane, row_bytes), ln.off, G);
    store_nt(make_rsrc(row + 2 * plane, row_bytes), ln.off, B);
}

// One band of rows [r0, r1) of one image for the wave's 256 columns.
template <bool EDGE>
__device__ __forceinline__ void run_band(const uint16_t* im, uint16_t* out, int H, int W, int r0,
                                         int r1, const Lane& ln) {
    const size_t plane = (size_t)H * (size_t)W;
    const uint32_t row_bytes = (uint32_t)W * 2u;
    auto fetch = [&](int rr) {
        return load_row(im + (size_t)mirror_row(rr, H) * (size_t)W, row_bytes, ln);
    };
    // Ring slot of row x: (x - r0 + 1) mod 3; the row loop is unrolled six
    // times, so the ring rotates by renaming and every row's parity is a
    // compile-time constant (r0 and the loop step are even). Two rows are in
    // flight: L[(x - r0 - 1) mod 2] holds row x until it is unpacked.
    Row U[3];
    U[0] = unpack<EDGE>(fetch(r0 - 1), ln);
    U[1] = unpack<EDGE>(fetch(r0), ln);
    Load L[2];
    L[0] = fetch(r0 + 1);
    L[1] = fetch(r0 + 2);  // r0 + 2 <= r1: bands have at least 2 rows
    for (int base = r0; base < r1; base += 6) {
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const int r = base + k;
            if (r >= r1) break;
            U[(k + 2) % 3] = unpack<EDGE>(L[k % 2], ln);  // row r + 1
            if (r + 3 <= r1) L[k % 2] = fetch(r + 3);
            finish_row((k & 1) == 0, U[k % 3], U[(k + 1) % 3], U[(k + 2) % 3],
                       out + (size_t)r * (size_t)W, plane, row_bytes, ln);
        }
    }
}

__global__ __launch_bounds__(256) void k_demosaic(const uint16_t* __restrict__ raw,
                                                  uint16_t* __restrict__ rgb, int32_t images,
                                                  int32_t H, int32_t W, int32_t band,
                                                  int32_t bands, int32_t col_waves) {
    const int lane = threadIdx.x & 63;
    // Wave-uniform (scalar) from here: the wave index and everything derived from it.
    const int wave =
        __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
    const int per_image = bands * col_waves;
    if (wave >= images * per_image) return;  // whole waves of the last block
    const int img = wave / per_image;
    const int rem = wave - img * per_image;
    const int bi = rem / col_waves;
    const int cw = rem - bi * col_waves;
    const int c0 = (cw * 64 + lane) * 4;
    Lane ln;
    ln.off = (uint32_t)c0 * 2u;
    ln.edge_off = lane == 0 ? ln.off - 4u : (lane == 63 ? ln.off + 8u : 0xfffffff0u);
    ln.at_start = c0 == 0;
    ln.at_end = c0 + 4 == W;
    const int r0 = bi * band;
    const int r1 = min(H, r0 + band);
    const size_t plane = (size_t)H * (size_t)W;
    const uint16_t* im = raw + (size_t)img * plane;
    uint16_t* out = rgb + (size_t)img * 3 * plane;
    if (cw == 0 || cw == col_waves - 1)
        run_band<true>(im, out, H, W, r0, r1, ln);
    else
        run_band<false>(im, out, H, W, r0, r1, ln);
}

}  // namespace

hipError_t launch_demosaic(const uint16_t* raw, int32_t images, int32_t H, int32_t W,
                           uint16_t* rgb, int cus, hipStream_t stream) {
    const int col_waves = (W / 4 + 63) / 64;
    // Long bands (few, long row streams) unless the launch is small: about 8
    // waves per CU over the launch, 12 when the whole launch is at most 64
    // rows per such wave (one 2048 x 2048 image: 6-row bands); 4 to 128 rows.
    // Measured on 16 images: 82.5 us at 128-row bands against 86 us at 32.
    if (cus <= 0) cus = 256;
    const int64_t col_total = (int64_t)images * col_waves;
    const int64_t work = (int64_t)H * col_total;  // wave-rows
    const int64_t target = (work <= (int64_t)64 * 8 * cus ? 12 : 8) * (int64_t)cus;
    int64_t band = (work + target - 1) / target;
    band = band < 4 ? 4 : (band > 128 ? 128 : band);
    band = (band + 1) & ~(int64_t)1;  // whole Bayer rows
    const int bands = (int)(((int64_t)H + band - 1) / band);
    const int64_t waves = col_total * bands;
    const int64_t blocks = (waves + 3) / 4;
    hipLaunchKernelGGL(k_demosaic, dim3((unsigned)blocks), dim3(256), 0, stream, raw, rgb, images,
                       H, W, (int)band, bands, col_waves);
    return hipGetLastError();
}

}  // namespace rc

using namespace rc;

extern "C" {

rc_status rc_demosaic(const uint16_t* raw, int32_t images, int32_t height, int32_t width,
                      uint16_t* rgb, hipStream_t stream) {
    if (images < 0 || height < 0 || width < 0) return RC_EINVAL;
    int64_t px = 0, n = 0;
    if (!mul_ok(height, width, &px) || !mul_ok(px, images, &n) || n > INT64_MAX / 8)
        return RC_EINVAL;
    if (n == 0) return RC_OK;
    if (height % 2 || width % 4 || height < 2 || width < 4) return RC_EINVAL;
    if (!raw || !rgb) return RC_EINVAL;
    if (((uintptr_t)raw | (uintptr_t)rgb) & 7u) return RC_EINVAL;
    if (overlaps(raw, (size_t)n * 2, rgb, (size_t)n * 6)) return RC_EINVAL;
    // Wave indices are 32-bit: images x bands x column waves < 2^31.
    if ((int64_t)images * (height / 2 + 1) * ((width / 4 + 63) / 64) >= ((int64_t)1 << 31))
        return RC_EINVAL;
    const DeviceInfo* di = current_device();
    if (!di) return RC_EHIP;
    hipError_t e = launch_demosaic(raw, images, height, width, rgb, di->cus, stream);
    return e == hipSuccess ? RC_OK : hip_fail(e);
}

}  // extern "C"
