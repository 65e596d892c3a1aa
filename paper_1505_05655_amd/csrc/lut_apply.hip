// Correction kernel (§I "Image Correction"): out[b][n][d] = lut[b][d][min(dn, L-1)].
//
// One workgroup per tile (band, strip of W detectors, chunk of lines). The
// raw LDS path stages the strip's W LUT rows into LDS level-major; the packed
// LDS path stages them as 2.5-bit step codes so strips are 6.4x wider; both
// then stream the chunk's lines through coalesced vector loads/stores. The
// L2 path gathers straight from the global LUT and orders tiles so that the
// CUs of one XCD share a strip whose LUT rows stay in that XCD's L2.
#include "device_ops.h"
#include "kernels.h"

namespace rc {

template <int VEC, int UNROLL, int NT, int MODE>
__global__ __launch_bounds__(1024) void k_apply(ApplyParams p) {
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
    const int W = 1 << p.log_strip;
    const int d0 = s * W;
    const int weff = min(W, p.detectors - d0);
    const int64_t n0 = (int64_t)c * p.chunk_lines;
    const int64_t n1 = min(p.lines, n0 + p.chunk_lines);
    apply_tile<VEC, UNROLL, NT, MODE>(p.dn, p.lut, p.out, p.lines, p.detectors, p.levels,
                                       p.log_strip, b, d0, weff, n0, n1, smem, p.lut_vec != 0);
}

typedef void (*ApplyKernel)(ApplyParams);

namespace {

// row[nontemporal * 3 + mode], mode = rc_path value (raw LDS, L2, packed LDS),
// nontemporal = 0 (none), 1 (loads and stores), 2 (stores only)
template <int VEC, int UNROLL>
void fill_row(ApplyKernel* row) {
    row[0] = k_apply<VEC, UNROLL, 0, kRaw>;
    row[1] = k_apply<VEC, UNROLL, 0, kGlobal>;
    row[2] = k_apply<VEC, UNROLL, 0, kPacked>;
    row[3] = k_apply<VEC, UNROLL, 1, kRaw>;
    row[4] = k_apply<VEC, UNROLL, 1, kGlobal>;
    row[5] = k_apply<VEC, UNROLL, 1, kPacked>;
    row[6] = k_apply<VEC, UNROLL, 2, kRaw>;
    row[7] = k_apply<VEC, UNROLL, 2, kGlobal>;
    row[8] = k_apply<VEC, UNROLL, 2, kPacked>;
}

// table[vec index][unroll index][nontemporal * 3 + mode]
struct Table {
    ApplyKernel k[3][3][9];
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
    }
};

const Table& table() {
    static const Table t;
    return t;
}

int vec_index(int vec) { return vec == 1 ? 0 : (vec == 2 ? 1 : 2); }
int unroll_index(int u) { return u == 4 ? 0 : (u == 8 ? 1 : 2); }

}  // namespace

hipError_t prepare_apply_kernels(size_t bytes, size_t* usable) {
    // A kernel's dynamic LDS limit is the CU's LDS minus its own static LDS
    // (e.g. the word __syncthreads_or reduces through).
    const Table& t = table();
    size_t worst_static = 0;
    for (int v = 0; v < 3; ++v)
        for (int u = 0; u < 3; ++u)
            for (int m = 0; m < 9; ++m) {
                if (m % 3 == kGlobal) continue;
                hipFuncAttributes attr;
                hipError_t e = hipFuncGetAttributes(&attr, (const void*)t.k[v][u][m]);
                if (e != hipSuccess) return e;
                worst_static = attr.sharedSizeBytes > worst_static ? attr.sharedSizeBytes
                                                                   : worst_static;
            }
    const size_t dyn = bytes > worst_static ? bytes - worst_static : 0;
    for (int v = 0; v < 3; ++v)
        for (int u = 0; u < 3; ++u)
            for (int m = 0; m < 9; ++m) {
                if (m % 3 == kGlobal) continue;
                hipError_t e = hipFuncSetAttribute((const void*)t.k[v][u][m],
                                                   hipFuncAttributeMaxDynamicSharedMemorySize,
                                                   (int)dyn);
                if (e != hipSuccess) return e;
            }
    *usable = dyn;
    return hipSuccess;
}

hipError_t launch_apply(const ApplyParams& p, const rc_plan& plan, size_t lds_bytes,
                        hipStream_t stream) {
    ApplyKernel k = table().k[vec_index(plan.vec)][unroll_index(plan.unroll)]
                             [plan.nontemporal * 3 + plan.path];
    hipLaunchKernelGGL(k, dim3((unsigned)p.ntiles), dim3((unsigned)plan.threads),
                       plan.path == RC_PATH_L2 ? 0 : lds_bytes, stream, p);
    return hipGetLastError();
}

}  // namespace rc
