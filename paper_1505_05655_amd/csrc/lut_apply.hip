// Correction kernel (§I "Image Correction"): out[b][n][d] = lut[b][d][min(dn, L-1)].
//
// One workgroup per tile (band, strip of detectors, chunk of lines). The raw
// LDS path stages the strip's LUT rows into LDS level-major; the packed and
// dense LDS paths stage them as 2.5-bit and 1.25-bit step codes, so strips
// are 6.4x and 12.8x wider (the dense blocks come from k_dense_encode's
// workspace, or are encoded by the tile); all then stream the chunk's lines
// (contiguous, or every k-th pass of the band) through coalesced vector
// loads/stores. The L2 path gathers straight from the global LUT and orders
// tiles so that the CUs of one XCD share a strip whose LUT rows stay in that
// XCD's L2.
#include "device_ops.h"
#include "kernels.h"

namespace rc {

// The dense mode runs at most 512 threads (its 160 KiB tile allows one
// workgroup per CU, two waves per SIMD): the tighter bound leaves it the
// registers to keep every pixel's LDS reads of a register set in flight.
template <int VEC, int UNROLL, int NT, int MODE>
__global__ __launch_bounds__(MODE == kDense ? kDenseMaxThreads : 1024) void k_apply(ApplyParams p) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int t = xcd_tile((int)blockIdx.x, (int)gridDim.x, p.xcds);
    int s, c, b;
    if (p.chunk_major) {
        c = t % p.chunks;
        const int r = t / p.chunks;
        s = r % p.strips;
        b = r / p.strips;
    } else {
        s = t % p.strips;
        const int r = t / p.strips;
        c = r % p.chunks;
        b = r / p.chunks;
    }
    int d0, weff;
    if (p.uneven) {
        const int64_t units = p.detectors / p.vec;
        const int u0 = (int)((int64_t)s * units / p.strips);
        const int u1 = (int)((int64_t)(s + 1) * units / p.strips);
        d0 = u0 * p.vec;
        weff = (u1 - u0) * p.vec;
    } else {
        const int W = 1 << p.log_strip;
        d0 = s * W;
        weff = min(W, p.detectors - d0);
    }
    // Line chunk c: contiguous lines, or (interleaved) every chunks-th pass
    // of the band's lines from pass c, so that the tiles of one strip read
    // neighbouring lines at the same time.
    int64_t n0 = 0, n1 = p.lines;
    int ci = 0, ck = 1;
    if (p.interleave) {
        ci = c;
        ck = p.chunks;
    } else {
        n0 = (int64_t)c * p.chunk_lines;
        n1 = min(p.lines, n0 + p.chunk_lines);
    }
    apply_tile<VEC, UNROLL, NT, MODE>(p.dn, p.lut, p.out, p.lines, p.detectors, p.levels,
                                       p.log_strip, b, d0, weff, n0, n1, smem, p.lut_vec != 0,
                                       p.dense != 0, p.pre_planes, p.pre_heads, ci, ck, p.threads);
}

// One thread per (row, 64-level block). Consecutive threads take the same
// block of consecutive rows: their output words are consecutive (output
// [band][block][detector]), and a wave's blocks are mostly of one kind
// (interior, run of 0 or run of L-1), so it rarely runs every branch of
// the encoder; each lane reads its block's 128 bytes as 16-byte loads.
__global__ __launch_bounds__(256) void k_dense_encode(const uint16_t* __restrict__ lut,
                                                      int64_t rows, int32_t detectors,
                                                      int32_t levels, uint64_t* planes,
                                                      int16_t* heads, int32_t vec16) {
    const int NB = (levels + 63) >> 6;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= rows * NB) return;
    const int64_t bands = rows / detectors;
    const int64_t per_block = bands * detectors;  // threads per block index
    const int blk = (int)(t / per_block);
    const int64_t row = t - (int64_t)blk * per_block;
    const int64_t b = row / detectors;
    const int64_t d = row - b * detectors;
    const size_t o = ((size_t)b * NB + (size_t)blk) * (size_t)detectors + (size_t)d;
    dense_encode_row_block(lut + (size_t)row * (size_t)levels, levels, blk, vec16 != 0,
                           planes + o, heads + o);
}

typedef void (*ApplyKernel)(ApplyParams);

namespace {

// row[policy * kModes + mode], mode = rc_path value (raw LDS, L2, packed
// LDS, dense LDS), policy = the plan's image cache policy (0..kPolicies-1)
constexpr int kModes = 4;

template <int VEC, int UNROLL, int NT>
void fill_policy(ApplyKernel* row) {
    row[NT * kModes + 0] = k_apply<VEC, UNROLL, NT, kRaw>;
    row[NT * kModes + 1] = k_apply<VEC, UNROLL, NT, kGlobal>;
    row[NT * kModes + 2] = k_apply<VEC, UNROLL, NT, kPacked>;
    row[NT * kModes + 3] = k_apply<VEC, UNROLL, NT, kDense>;
}

template <int VEC, int UNROLL>
void fill_row(ApplyKernel* row) {
    fill_policy<VEC, UNROLL, 0>(row);
    fill_policy<VEC, UNROLL, 1>(row);
    fill_policy<VEC, UNROLL, 2>(row);
    fill_policy<VEC, UNROLL, 3>(row);
    fill_policy<VEC, UNROLL, 4>(row);
    fill_policy<VEC, UNROLL, 5>(row);
    static_assert(kPolicies == 6, "one fill_policy per cache policy");
}

constexpr int kRow = kPolicies * kModes;

// table[vec index][unroll index][policy * kModes + mode]
struct Table {
    ApplyKernel k[4][3][kRow];
    Table() {
        fill_row<1, 4>(k[0][0]);
        fill_row<1, 8>(k[0][1]);
        fill_row<1, 16>(k[0][2]);
        fill_row<2, 4>(k[1][0]);
        fill_row<2, 8>(k[1][1]);
        fill_row<2, 16>(k[1][2]);
        fill_row<4, 4>(k[2][0]);
        fill_row<4, 8>(k[2][1]);
        fill_row<4, 16>(k[2][2]);
        fill_row<8, 4>(k[3][0]);
        // 8 pixels x 8 or 16 lines per register set spill registers: not
        // built, and check_plan rejects them (8 x 4 holds as many pixels per
        // set as 4 x 8).
        for (int m = 0; m < kRow; ++m) k[3][1][m] = k[3][2][m] = nullptr;
    }
};

const Table& table() {
    static const Table t;
    return t;
}

int vec_index(int vec) { return vec == 1 ? 0 : (vec == 2 ? 1 : (vec == 4 ? 2 : 3)); }
int unroll_index(int u) { return u == 4 ? 0 : (u == 8 ? 1 : 2); }

}  // namespace

hipError_t prepare_apply_kernels(size_t bytes, size_t* usable) {
    // A kernel's dynamic LDS limit is the CU's LDS minus its own static LDS
    // (none in these kernels; the dense mode relies on that).
    const Table& t = table();
    size_t worst_static = 0;
    for (int v = 0; v < 4; ++v)
        for (int u = 0; u < 3; ++u)
            for (int m = 0; m < kRow; ++m) {
                if (m % kModes == kGlobal || !t.k[v][u][m]) continue;
                hipFuncAttributes attr;
                hipError_t e = hipFuncGetAttributes(&attr, (const void*)t.k[v][u][m]);
                if (e != hipSuccess) return e;
                // The dense decode addresses LDS from byte 0, which is where
                // the dynamic LDS starts only with no static LDS.
                if (m % kModes == kDense && attr.sharedSizeBytes != 0) return hipErrorInvalidImage;
                worst_static = attr.sharedSizeBytes > worst_static ? attr.sharedSizeBytes
                                                                   : worst_static;
            }
    const size_t dyn = bytes > worst_static ? bytes - worst_static : 0;
    for (int v = 0; v < 4; ++v)
        for (int u = 0; u < 3; ++u)
            for (int m = 0; m < kRow; ++m) {
                if (m % kModes == kGlobal || !t.k[v][u][m]) continue;
                hipError_t e = hipFuncSetAttribute((const void*)t.k[v][u][m],
                                                   hipFuncAttributeMaxDynamicSharedMemorySize,
                                                   (int)dyn);
                if (e != hipSuccess) return e;
            }
    *usable = dyn;
    return hipSuccess;
}

hipError_t launch_dense_encode(const uint16_t* lut, int32_t bands, int32_t detectors,
                               int32_t levels, uint64_t* planes, int16_t* heads,
                               hipStream_t stream) {
    const int64_t rows = (int64_t)bands * detectors;
    const int64_t items = rows * ((levels + 63) / 64);
    if (items <= 0) return hipSuccess;
    const int vec16 = (levels % 8 == 0 && ((uintptr_t)lut & 15u) == 0) ? 1 : 0;
    hipLaunchKernelGGL(k_dense_encode, dim3((unsigned)((items + 255) / 256)), dim3(256), 0, stream,
                       lut, rows, detectors, levels, planes, heads, vec16);
    return hipGetLastError();
}

hipError_t launch_apply(const ApplyParams& p, const rc_plan& plan, size_t lds_bytes,
                        hipStream_t stream) {
    ApplyKernel k = table().k[vec_index(plan.vec)][unroll_index(plan.unroll)]
                             [plan.nontemporal * kModes + plan.path];
    if (!k) return hipErrorInvalidValue;  // combinations check_plan rejects
    hipLaunchKernelGGL(k, dim3((unsigned)p.ntiles), dim3((unsigned)p.block),
                       plan.path == RC_PATH_L2 ? 0 : lds_bytes, stream, p);
    return hipGetLastError();
}

}  // namespace rc
