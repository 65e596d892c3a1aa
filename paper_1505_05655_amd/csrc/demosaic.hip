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
// registers: each row is loaded once, the next row's load is in flight while
// the current row is computed. The left and right neighbour columns come from the adjacent lanes
// by lane shuffles; only the two lanes at a wave's edge load them. No LDS.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"
#include "rc.h"
#include "runtime.h"

namespace rc {
namespace {

struct Row {
    uint32_t v[4];   // columns c0 .. c0+3
    uint32_t w, e;   // columns c0-1 and c0+4 (mirrored at the image edges)
};

__device__ __forceinline__ int mirror_row(int r, int H) {
    return r < 0 ? -r : (r >= H ? 2 * (H - 1) - r : r);
}

struct RawRow {
    uint2 q;          // the 4 samples, two per dword
    uint32_t edge;    // column c0-1 (lane 0) or c0+4 (lane 63), if needed
};

__device__ __forceinline__ RawRow load_row(const uint16_t* im, int W, int r, int c0, bool valid,
                                           int lane) {
    RawRow x;
    x.q = make_uint2(0u, 0u);
    x.edge = 0u;
    if (valid) {
        const uint16_t* p = im + (size_t)r * (size_t)W;
        x.q = *(const uint2*)(p + c0);
        if (lane == 0 && c0 > 0) x.edge = p[c0 - 1];
        if (lane == 63 && c0 + 4 < W) x.edge = p[c0 + 4];
    }
    return x;
}

__device__ __forceinline__ Row unpack(const RawRow& x, int c0, int W, int lane) {
    Row r;
    r.v[0] = x.q.x & 0xffffu;
    r.v[1] = x.q.x >> 16;
    r.v[2] = x.q.y & 0xffffu;
    r.v[3] = x.q.y >> 16;
    const uint32_t from_left = (uint32_t)__shfl_up((int)r.v[3], 1, 64);
    const uint32_t from_right = (uint32_t)__shfl_down((int)r.v[0], 1, 64);
    // Column c0-1: mirrored to column 1 at the left edge.
    r.w = c0 == 0 ? r.v[1] : (lane == 0 ? x.edge : from_left);
    // Column c0+4: mirrored to column W-2 at the right edge.
    r.e = c0 + 4 == W ? r.v[2] : (lane == 63 ? x.edge : from_right);
    return r;
}

// Neighbour k of column j (0..3) in a row: k = -1 left, 0 self, +1 right.
__device__ __forceinline__ uint32_t at(const Row& r, int j, int k) {
    const int t = j + k;
    return t < 0 ? r.w : (t > 3 ? r.e : r.v[t]);
}

__global__ __launch_bounds__(256) void k_demosaic(const uint16_t* __restrict__ raw,
                                                  uint16_t* __restrict__ rgb, int32_t images,
                                                  int32_t H, int32_t W, int32_t band,
                                                  int32_t bands, int32_t col_waves) {
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

    Row P = unpack(load_row(im, W, mirror_row(r0 - 1, H), c0, valid, lane), c0, W, lane);
    Row C = unpack(load_row(im, W, r0, c0, valid, lane), c0, W, lane);
    RawRow nx = load_row(im, W, mirror_row(r0 + 1, H), c0, valid, lane);
    for (int r = r0; r < r1; ++r) {
        const Row N = unpack(nx, c0, W, lane);
        // The row after next is loaded while this row is computed.
        nx = load_row(im, W, mirror_row(r + 2, H), c0, valid && r + 1 < r1, lane);
        uint32_t R[4], G[4], B[4];
        const bool red_row = (r & 1) == 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t self = C.v[j];
            const uint32_t hor = at(C, j, -1) + at(C, j, 1);
            const uint32_t ver = P.v[j] + N.v[j];
            const uint32_t diag = at(P, j, -1) + at(P, j, 1) + at(N, j, -1) + at(N, j, 1);
            const uint32_t cross = (hor + ver + 2) >> 2;
            const uint32_t dg = (diag + 2) >> 2;
            const uint32_t h2 = (hor + 1) >> 1, v2 = (ver + 1) >> 1;
            if (red_row) {
                if ((j & 1) == 0) {  // red pixel (c0 is even)
                    R[j] = self;
                    G[j] = cross;
                    B[j] = dg;
                } else {             // green pixel in a red row
                    R[j] = h2;
                    G[j] = self;
                    B[j] = v2;
                }
            } else {
                if ((j & 1) == 0) {  // green pixel in a blue row
                    R[j] = v2;
                    G[j] = self;
                    B[j] = h2;
                } else {             // blue pixel
                    R[j] = dg;
                    G[j] = cross;
                    B[j] = self;
                }
            }
        }
        if (valid) {
            const size_t o = (size_t)r * (size_t)W + (size_t)c0;
            // Non-temporal: the planes are written once and not read back here.
            uint32_t* q = (uint32_t*)(out + o);
            __builtin_nontemporal_store(R[0] | (R[1] << 16), q);
            __builtin_nontemporal_store(R[2] | (R[3] << 16), q + 1);
            q = (uint32_t*)(out + plane + o);
            __builtin_nontemporal_store(G[0] | (G[1] << 16), q);
            __builtin_nontemporal_store(G[2] | (G[3] << 16), q + 1);
            q = (uint32_t*)(out + 2 * plane + o);
            __builtin_nontemporal_store(B[0] | (B[1] << 16), q);
            __builtin_nontemporal_store(B[2] | (B[3] << 16), q + 1);
        }
        P = C;
        C = N;
    }
}

}  // namespace

hipError_t launch_demosaic(const uint16_t* raw, int32_t images, int32_t H, int32_t W,
                           uint16_t* rgb, int cus, hipStream_t stream) {
    const int col_waves = (W / 4 + 63) / 64;
    // Bands of rows short enough for about 32 waves per CU over the launch,
    // long enough that the two halo rows of a band cost little (<= 64 rows).
    const int64_t target = (int64_t)32 * (cus > 0 ? cus : 256);
    const int64_t col_total = (int64_t)images * col_waves;
    int64_t band = ((int64_t)H * col_total + target - 1) / target;
    band = band < 4 ? 4 : (band > 64 ? 64 : band);
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
