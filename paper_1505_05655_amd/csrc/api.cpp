// C-ABI entry points of the plain path: validation, plan choice, launch.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <mutex>

#include "device_ops.h"
#include "kernels.h"
#include "rc.h"
#include "runtime.h"

namespace rc {

namespace {

thread_local int32_t t_last_hip = 0;

constexpr int kMaxDevices = 64;
DeviceInfo g_info[kMaxDevices];
bool g_ready[kMaxDevices];
std::mutex g_mu;

int ilog2(int64_t x) {
    int r = 0;
    while (((int64_t)1 << (r + 1)) <= x) ++r;
    return r;
}

bool is_pow2(int64_t x) { return x > 0 && (x & (x - 1)) == 0; }

}  // namespace

rc_status hip_fail(hipError_t e) {
    t_last_hip = (int32_t)e;
    return RC_EHIP;
}

const DeviceInfo* current_device(int* dev_out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        hip_fail(e);
        return nullptr;
    }
    if (dev < 0 || dev >= kMaxDevices) {
        hip_fail(hipErrorInvalidDevice);
        return nullptr;
    }
    if (dev_out) *dev_out = dev;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ready[dev]) {
        hipDeviceProp_t prop;
        e = hipGetDeviceProperties(&prop, dev);
        if (e != hipSuccess) {
            hip_fail(e);
            return nullptr;
        }
        DeviceInfo& di = g_info[dev];
        di.cus = prop.multiProcessorCount;
        di.lds = prop.sharedMemPerBlock;
        if (prop.sharedMemPerBlockOptin > di.lds) di.lds = prop.sharedMemPerBlockOptin;
        di.lds_per_cu = prop.maxSharedMemoryPerMultiProcessor ? prop.maxSharedMemoryPerMultiProcessor
                                                              : di.lds;
        di.arch = prop.gcnArchName;
        const size_t colon = di.arch.find(':');
        if (colon != std::string::npos) di.arch.resize(colon);
        di.hbm_bytes = prop.totalGlobalMem;
        int x = 1;
        if (hipDeviceGetAttribute(&x, hipDeviceAttributeNumberOfXccs, dev) != hipSuccess || x < 1)
            x = 1;
        di.xcds = x;
        size_t usable = 0;
        e = prepare_apply_kernels(di.lds, &usable);
        if (e != hipSuccess) {
            hip_fail(e);
            return nullptr;
        }
        di.lds = usable;
        g_ready[dev] = true;
    }
    return &g_info[dev];
}

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return na && nb && x < y + nb && y < x + na;
}

bool mul_ok(int64_t a, int64_t b, int64_t* r) { return !__builtin_mul_overflow(a, b, r); }

int max_vec(const uint16_t* dn, const uint16_t* out, int32_t detectors, int cap) {
    const uintptr_t al = (uintptr_t)dn | (uintptr_t)out;
    if (cap >= 8 && detectors % 8 == 0 && (al & 15u) == 0) return 8;
    if (cap >= 4 && detectors % 4 == 0 && (al & 7u) == 0) return 4;
    if (detectors % 2 == 0 && (al & 3u) == 0) return 2;
    return 1;
}

int plan_slots(const rc_plan& plan, size_t lds_bytes, const DeviceInfo& di) {
    int per_cu = std::max(1, 2048 / std::max(64, (int)plan.threads));
    if (plan.path != RC_PATH_L2 && lds_bytes) {
        per_cu = std::min<int>(per_cu, (int)(di.lds_per_cu / lds_bytes));
    }
    return std::max(1, per_cu) * std::max(1, di.cus);
}

int64_t max_chunk_lines(int32_t detectors, int32_t threads, int32_t unroll) {
    // Tile pixels are addressed with 32-bit buffer offsets: a tile's lines
    // plus up to two passes of overshoot must stay below 2^31 bytes.
    return ((int64_t)1 << 31) / (2 * (int64_t)std::max(detectors, 1)) -
           2 * (int64_t)threads * unroll;
}

size_t plan_lds_bytes(int path, int strip, int levels) {
    if (path == RC_PATH_LDS) return (size_t)strip * (size_t)levels * 2;
    if (path == RC_PATH_PACKED) return packed_lds_bytes(strip, levels);
    if (path == RC_PATH_DENSE) return dense_lds_bytes(strip, levels);
    return 0;
}

// Widest power-of-two strip (<= 1024 detectors) whose LDS tile fits `budget`.
int widest_strip(int path, int levels, size_t budget) {
    int W = 1024;
    while (W > 1 && plan_lds_bytes(path, W, levels) > budget) W >>= 1;
    return W;
}

// Legacy launch shape: power-of-two strips of W detectors, the line chunk
// count sized for about two rounds of resident tiles. Used for the L2 path
// (LUT rows too long for any useful LDS strip) and small scenes.
void pow2_plan(int64_t lines, int32_t detectors, int32_t bands, int32_t levels, int vmax,
               const DeviceInfo& di, rc_plan* plan) {
    rc_plan p;
    std::memset(&p, 0, sizeof(p));
    const size_t budget = std::min<size_t>(di.lds ? di.lds : 65536, 80 * 1024);
    const int path_lds = levels >= 512 ? RC_PATH_PACKED : RC_PATH_LDS;
    const int W = std::min(256, widest_strip(path_lds, levels, budget));
    const int64_t dcap = std::max<int64_t>(1, (int64_t)1 << (ilog2(detectors) +
                                                              (is_pow2(detectors) ? 0 : 1)));
    if (W >= 16) {
        p.path = path_lds;
        p.strip = (int)std::min<int64_t>(W, dcap);
    } else {
        p.path = RC_PATH_L2;
        p.strip = (int)std::min<int64_t>(64, dcap);
    }
    p.vec = std::min(std::min(vmax, 4), p.strip >= 128 ? 4 : 2);
    while (p.vec > p.strip) p.vec >>= 1;
    p.threads = 512;
    p.unroll = 8;
    p.xcd_remap = 1;
    p.nontemporal = p.strip >= 256 ? 2 : 0;
    const size_t lds_bytes = plan_lds_bytes(p.path, p.strip, levels);
    const int slots = plan_slots(p, lds_bytes, di);
    const int64_t strips = (detectors + p.strip - 1) / p.strip;
    const int64_t base = std::max<int64_t>(1, (int64_t)bands * strips);
    const int64_t cap = std::max<int64_t>(1, max_chunk_lines(detectors, p.threads, p.unroll));
    const int64_t kmin = (lines + cap - 1) / cap;
    // Wide strips stream fast enough per workgroup that one tile per strip is
    // best once most CUs get one; narrower strips need about two waves of
    // resident tiles to keep enough lines in flight.
    int64_t k = (p.strip >= 256 && base * 10 >= (int64_t)di.cus * 6)
                    ? 1
                    : (2 * (int64_t)slots + base - 1) / base;
    k = std::max(k, kmin);
    if (p.path == RC_PATH_L2) {
        k = std::max<int64_t>(k, 32);
    } else {
        // Re-staging cost of k chunks relative to the image bytes.
        const int64_t kcap = std::max<int64_t>(1, (int64_t)(0.2 * 2.0 * (double)lines /
                                                            (double)levels));
        k = std::max<int64_t>(kmin, std::min(k, kcap));
    }
    k = std::min<int64_t>(k, std::max<int64_t>(1, lines));
    p.chunk_lines = (int32_t)std::min<int64_t>((lines + k - 1) / k, INT32_MAX);
    *plan = p;
}

bool balanced_tiling(int64_t lines, int32_t detectors, int32_t bands, int vec, int wmax,
                     int64_t target, int32_t threads, int32_t unroll, int32_t* strips_out,
                     int32_t* strip_out, int32_t* chunk_lines_out) {
    const int64_t units = detectors / std::max(vec, 1);
    if (vec < 1 || wmax < vec || units < 1 || lines < 1 || bands < 1) return false;
    target = std::max<int64_t>(1, target);
    const int64_t per_strip = wmax / vec;                      // units per strip at most
    const int64_t smin = (units + per_strip - 1) / per_strip;  // strips needed to fit LDS
    const int64_t sfill = std::max<int64_t>(1, target / bands);
    const int64_t swide = std::max<int64_t>(1, (int64_t)detectors / 64);  // >= 64 detectors
    int64_t strips = std::max(smin, std::min(sfill, swide));
    strips = std::min(strips, units);
    int64_t k = std::max<int64_t>(1, target / ((int64_t)bands * strips));
    const int64_t cap = max_chunk_lines(detectors, threads, unroll);
    if (cap < 1) return false;
    k = std::max(k, (lines + cap - 1) / cap);
    k = std::min<int64_t>(k, lines);
    const int64_t widest = vec * ((units + strips - 1) / strips);
    int W = 1;
    while (W < widest) W <<= 1;
    if (strips > INT32_MAX || (lines + k - 1) / k > INT32_MAX) return false;
    *strips_out = (int32_t)strips;
    *strip_out = W;
    *chunk_lines_out = (int32_t)((lines + k - 1) / k);
    return true;
}

// Default launch shape (no tuning), from measurements on MI355X. Two tilings:
//  - power-of-two strips of W detectors in an 80 KiB LDS tile (W = 256 for
//    L <= 2048: 512-byte line segments), one line chunk when that already
//    gives most CUs a tile (pow2_plan);
//  - when the CU share of the detectors (bands x detectors / CUs) is wider
//    than that W (long LUT rows: W = 64 at L = 4096), one tile per CU: each
//    band cut into strips of equal width so that the tile count matches the
//    CU count, the LUT strip in a 160 KiB tile staged once, 256 threads
//    (one wave per SIMD, 2 pixels x 8 lines per lane and register set, no
//    idle lanes), which keeps the fewest lines in flight per CU for the bytes
//    it moves: more threads per CU made the L2 re-fetch the partial cache
//    lines that neighbouring strips share (measured 1.7x the reads with 1024).
void default_plan(int64_t lines, int32_t detectors, int32_t bands, int32_t levels, int vmax,
                  const DeviceInfo& di, rc_plan* plan) {
    rc_plan legacy;
    pow2_plan(lines, detectors, bands, levels, vmax, di, &legacy);
    const int64_t cus = std::max(1, di.cus);
    const size_t cu_budget = std::min(di.lds ? di.lds : (size_t)65536,
                                      di.lds_per_cu ? di.lds_per_cu : (size_t)65536);
    // Long LUT rows (2048 <= L <= 8192) of a large scene: dense strips of up
    // to 256 detectors (512-byte line segments) in one 160 KiB tile per CU,
    // 512 threads, line chunks so that about one tile per CU runs. Each tile
    // encodes its strip (W x L entries) before it streams, so only when a
    // tile has at least 4 L lines to stream.
    const int wdense = std::min(256, widest_strip(RC_PATH_DENSE, levels, cu_budget));
    const int64_t dstrips = (detectors + wdense - 1) / std::max(wdense, 1);
    const int64_t dtiles = std::max<int64_t>(1, cus / std::max<int64_t>(1, bands * dstrips));
    if (levels >= 2048 && levels <= kDenseMaxLevels && wdense >= 64 && detectors >= 64 &&
        lines / dtiles >= 4 * (int64_t)levels) {
        rc_plan p;
        std::memset(&p, 0, sizeof(p));
        p.path = RC_PATH_DENSE;
        const int64_t dcap = (int64_t)1 << (ilog2(detectors) + (is_pow2(detectors) ? 0 : 1));
        p.strip = (int)std::min<int64_t>(wdense, dcap);
        p.vec = std::min(vmax, 4);
        p.threads = 512;
        p.unroll = 8;
        p.xcd_remap = 1;
        p.nontemporal = 0;
        const int64_t strips = (detectors + p.strip - 1) / p.strip;
        const int64_t cap = std::max<int64_t>(1, max_chunk_lines(detectors, p.threads, p.unroll));
        int64_t k = std::max<int64_t>(1, cus / std::max<int64_t>(1, (int64_t)bands * strips));
        k = std::max(k, (lines + cap - 1) / cap);
        k = std::min<int64_t>(k, std::max<int64_t>(1, lines));
        p.chunk_lines = (int32_t)std::min<int64_t>((lines + k - 1) / k, INT32_MAX);
        *plan = p;
        return;
    }
    const double share = (double)bands * (double)detectors / (double)cus;
    // One tile per CU stages a whole strip with few waves: worth it only when
    // the strip then streams many lines (at least 4 L).
    if (legacy.path == RC_PATH_L2 || share <= (double)legacy.strip ||
        lines < 4 * (int64_t)levels) {
        *plan = legacy;
        return;
    }
    const int path_lds = levels >= 512 ? RC_PATH_PACKED : RC_PATH_LDS;
    const size_t budget = std::min(di.lds ? di.lds : (size_t)65536,
                                   di.lds_per_cu ? di.lds_per_cu : (size_t)65536);
    const int wmax = widest_strip(path_lds, levels, budget);
    rc_plan p;
    std::memset(&p, 0, sizeof(p));
    p.path = path_lds;
    p.vec = std::min(vmax, 2);
    p.threads = 256;
    p.unroll = 8;
    p.xcd_remap = 1;
    p.nontemporal = 0;
    p.lane_map = 1;
    if (wmax < 16 || !balanced_tiling(lines, detectors, bands, p.vec, wmax, cus, p.threads,
                                      p.unroll, &p.strips, &p.strip, &p.chunk_lines)) {
        *plan = legacy;
        return;
    }
    *plan = p;
}

rc_status check_plan(const rc_plan& plan, int64_t lines, int32_t detectors, int32_t bands,
                     int32_t levels, int vmax, const DeviceInfo& di, ApplyParams* p,
                     size_t* lds_bytes) {
    if (plan.path != RC_PATH_LDS && plan.path != RC_PATH_L2 && plan.path != RC_PATH_PACKED &&
        plan.path != RC_PATH_DENSE)
        return RC_EINVAL;
    if (plan.path == RC_PATH_DENSE && levels > kDenseMaxLevels) return RC_EINVAL;
    if (plan.path == RC_PATH_DENSE && plan.threads > kDenseMaxThreads) return RC_EINVAL;
    if (!is_pow2(plan.strip) || plan.strip > 1024) return RC_EINVAL;
    if (plan.vec != 1 && plan.vec != 2 && plan.vec != 4 && plan.vec != 8) return RC_EINVAL;
    if (plan.vec > vmax || plan.strip < plan.vec) return RC_EINVAL;
    if (plan.threads != 256 && plan.threads != 512 && plan.threads != 1024) return RC_EINVAL;
    if (plan.unroll != 4 && plan.unroll != 8 && plan.unroll != 16) return RC_EINVAL;
    if (plan.vec == 8 && plan.unroll != 4) return RC_EINVAL;  // would spill registers
    if (plan.chunk_lines < 1) return RC_EINVAL;
    if (plan.nontemporal < 0 || plan.nontemporal >= kPolicies) return RC_EINVAL;
    if (plan.lane_map < 0 || plan.lane_map > 1) return RC_EINVAL;
    if (plan.xcd_remap < 0 || plan.xcd_remap > 1) return RC_EINVAL;
    if (plan.strip / plan.vec > plan.threads) return RC_EINVAL;
    const size_t bytes = plan_lds_bytes(plan.path, plan.strip, levels);
    if (bytes > di.lds) return RC_EINVAL;
    if (plan.chunk_lines > max_chunk_lines(detectors, plan.threads, plan.unroll)) return RC_EINVAL;
    if (plan.strips < 0) return RC_EINVAL;
    int64_t strips = (detectors + (int64_t)plan.strip - 1) / plan.strip;
    if (plan.strips > 0) {
        // vec divides detectors (vec <= vmax); strips of whole vec units, the
        // widest ceil(units / strips) units, at most W detectors.
        const int64_t units = detectors / plan.vec;
        if (plan.strips > units) return RC_EINVAL;
        if (plan.vec * ((units + plan.strips - 1) / plan.strips) > plan.strip) return RC_EINVAL;
        strips = plan.strips;
    }
    const int64_t chunks = (lines + plan.chunk_lines - 1) / plan.chunk_lines;
    int64_t tiles = 0;
    if (!mul_ok((int64_t)bands * strips, chunks, &tiles)) return RC_EINVAL;
    // A tile alone on its CU stages its strip with more waves than stream:
    // packing a 256 x 1024 strip with 4 waves (one per SIMD) is bound by
    // instruction issue (49 us on the 4 x 12000 x 12000 scene, against 31 us
    // with 16 waves); streaming with the plan's 256 threads stays faster than
    // with 1024 (0.509 against 0.525 ms). The extra waves wait at the tile's
    // barriers while the others stream.
    int block = plan.threads;
    if (di.cus > 0 && tiles <= di.cus) {
        if (plan.path == RC_PATH_LDS || plan.path == RC_PATH_PACKED) block = 1024;
        if (plan.path == RC_PATH_DENSE) block = kDenseMaxThreads;
    }
    if (tiles * block >= ((int64_t)1 << 32) || tiles > INT32_MAX) return RC_EINVAL;
    p->threads = plan.threads;
    p->block = std::max(block, plan.threads);
    p->pre_planes = nullptr;
    p->pre_heads = nullptr;
    p->lines = lines;
    p->detectors = detectors;
    p->levels = levels;
    p->bands = bands;
    p->log_strip = ilog2(plan.strip);
    p->strips = (int32_t)strips;
    p->uneven = plan.strips > 0 ? 1 : 0;
    p->vec = plan.vec;
    p->dense = plan.lane_map;
    p->chunks = (int32_t)chunks;
    p->chunk_lines = plan.chunk_lines;
    p->ntiles = (int32_t)tiles;
    p->xcds = plan.xcd_remap ? di.xcds : 1;
    p->chunk_major = plan.path == RC_PATH_L2 ? 1 : 0;
    // LDS tiles interleave their line chunks pass by pass (measured on the
    // 3 x 50000 x 6000 scene: the tiles of neighbouring strips and chunks
    // then stream neighbouring lines together, 3 % faster than contiguous
    // chunks) when a whole band, plus the prefetch overshoot of a tile that
    // steps `chunks` passes at a time, stays within the 32-bit offsets.
    p->interleave = (plan.path != RC_PATH_L2 && chunks > 1 &&
                     lines + 2 * (chunks - 1) * (int64_t)plan.threads * plan.unroll <=
                         max_chunk_lines(detectors, plan.threads, plan.unroll))
                        ? 1 : 0;
    *lds_bytes = bytes;
    return RC_OK;
}

namespace {

// Shape and pointer validation shared by rc_correct and rc_correct_plan.
rc_status validate_correct(const uint16_t* dn, const uint16_t* lut, int64_t lines,
                           int32_t detectors, int32_t bands, int32_t levels, const uint16_t* out,
                           bool* empty) {
    *empty = false;
    if (lines < 0 || detectors < 0 || bands < 0) return RC_EINVAL;
    if (levels < RC_LEVELS_MIN || levels > RC_LEVELS_MAX) return RC_EINVAL;
    int64_t px = 0, lut_n = 0, bytes = 0;
    if (!mul_ok(lines, detectors, &px) || !mul_ok(px, bands, &px) || !mul_ok(px, 2, &bytes))
        return RC_EINVAL;
    if (!mul_ok((int64_t)bands * detectors, levels, &lut_n) || !mul_ok(lut_n, 2, &lut_n))
        return RC_EINVAL;
    if (px == 0) {
        *empty = true;
        return RC_OK;
    }
    if (!dn || !lut || !out) return RC_EINVAL;
    if (((uintptr_t)dn | (uintptr_t)lut | (uintptr_t)out) & 1u) return RC_EINVAL;
    if (dn != out && overlaps(dn, (size_t)bytes, out, (size_t)bytes)) return RC_EINVAL;
    if (overlaps(lut, (size_t)lut_n, out, (size_t)bytes)) return RC_EINVAL;
    return RC_OK;
}

}  // namespace

bool ws_path(int32_t levels) { return levels >= 2048 && levels <= kDenseMaxLevels; }

size_t dense_ws_bytes(int32_t detectors, int32_t bands, int32_t levels) {
    const size_t n = (size_t)bands * (size_t)((levels + 63) / 64) * (size_t)detectors;
    return ((n * 8 + 255) & ~(size_t)255) + ((n * 2 + 255) & ~(size_t)255);
}

// Plan of the pre-encoded dense correction (measured on the 3 x 50000 x
// 6000, L = 4096 scene): strips of at most 256 detectors (line segments of
// up to 512 bytes), cut in equal widths so that bands x strips x line chunks
// comes close to the CU count with the fewest chunks that allow it (each
// chunk copies its strip's encoded blocks, 160 KiB, nothing to encode), one
// 160 KiB tile per CU, 256 threads with 8 pixels (16 bytes) x 4 lines per
// lane and register set, lanes packed without gaps.
void ws_plan(int64_t lines, int32_t detectors, int32_t bands, int32_t levels, int vmax,
             const DeviceInfo& di, rc_plan* plan) {
    const size_t cu_budget = std::min(di.lds ? di.lds : (size_t)65536,
                                      di.lds_per_cu ? di.lds_per_cu : (size_t)65536);
    rc_plan p;
    std::memset(&p, 0, sizeof(p));
    p.path = RC_PATH_DENSE;
    p.vec = std::min(vmax, 8);
    p.threads = 256;
    p.unroll = p.vec == 8 ? 4 : 8;
    p.xcd_remap = 1;
    p.lane_map = 1;
    const int wmax = std::min(256, widest_strip(RC_PATH_DENSE, levels, cu_budget));
    const int64_t cus = std::max(1, di.cus);
    const int64_t units = detectors / p.vec;
    const int64_t per = std::max(1, wmax / p.vec);
    const int64_t smin = std::max<int64_t>(1, (units + per - 1) / per);
    int64_t k = std::max<int64_t>(1, cus / std::max<int64_t>(1, (int64_t)bands * smin));
    const int64_t cap = std::max<int64_t>(1, max_chunk_lines(detectors, p.threads, p.unroll));
    k = std::max(k, (lines + cap - 1) / cap);
    k = std::min<int64_t>(k, std::max<int64_t>(1, lines));
    int64_t strips = std::max(smin, cus / std::max<int64_t>(1, (int64_t)bands * k));
    strips = std::min(strips, units);
    const int64_t widest = p.vec * ((units + strips - 1) / strips);
    int W = 1;
    while (W < widest) W <<= 1;
    p.strip = W;
    p.strips = (int32_t)strips;
    p.chunk_lines = (int32_t)std::min<int64_t>((lines + k - 1) / k, INT32_MAX);
    *plan = p;
}

namespace {

rc_status run_correct(const uint16_t* dn, const uint16_t* lut, int64_t lines, int32_t detectors,
                      int32_t bands, int32_t levels, uint16_t* out, const rc_plan* forced,
                      hipStream_t stream, void* ws = nullptr, size_t ws_bytes = 0,
                      bool pre_encoded = false) {
    bool empty = false;
    rc_status st = validate_correct(dn, lut, lines, detectors, bands, levels, out, &empty);
    if (st != RC_OK || empty) return st;
    const bool use_ws = ws != nullptr && ws_path(levels);
    uint64_t* planes = nullptr;
    int16_t* heads = nullptr;
    if (use_ws) {
        // The workspace holds the LUT's dense encoding: it may overlap none
        // of the call's other buffers.
        const size_t need = dense_ws_bytes(detectors, bands, levels);
        if (ws_bytes < need || ((uintptr_t)ws & 255u)) return RC_EINVAL;
        const size_t img = (size_t)lines * (size_t)detectors * (size_t)bands * 2;
        const size_t lut_b = (size_t)bands * (size_t)detectors * (size_t)levels * 2;
        if (overlaps(ws, need, dn, img) || overlaps(ws, need, out, img) ||
            overlaps(ws, need, lut, lut_b))
            return RC_EINVAL;
        const size_t n = (size_t)bands * (size_t)((levels + 63) / 64) * (size_t)detectors;
        planes = (uint64_t*)ws;
        heads = (int16_t*)((char*)ws + ((n * 8 + 255) & ~(size_t)255));
    }
    const DeviceInfo* di = current_device();
    if (!di) return RC_EHIP;
    const int vmax = max_vec(dn, out, detectors, 8);
    rc_plan plan;
    if (forced) {
        plan = *forced;
    } else if (use_ws) {
        ws_plan(lines, detectors, bands, levels, vmax, *di, &plan);
    } else if (!tuned_plan(lines, detectors, bands, levels, vmax, *di, &plan)) {
        default_plan(lines, detectors, bands, levels, vmax, *di, &plan);
    }
    if (use_ws && plan.path != RC_PATH_DENSE) return RC_EINVAL;
    ApplyParams p{};
    size_t lds_bytes = 0;
    st = check_plan(plan, lines, detectors, bands, levels, vmax, *di, &p, &lds_bytes);
    if (st != RC_OK) return st;
    p.dn = dn;
    p.lut = lut;
    p.out = out;
    p.lut_vec = (levels % 8 == 0 && ((uintptr_t)lut & 15u) == 0) ? 1 : 0;
    if (use_ws) {
        if (!pre_encoded) {
            hipError_t e = launch_dense_encode(lut, bands, detectors, levels, planes, heads, stream);
            if (e != hipSuccess) return hip_fail(e);
        }
        p.pre_planes = planes;
        p.pre_heads = heads;
    }
    // When the tiles fit in a few rounds of one tile per CU, cap the tiles
    // resident per CU at ceil(tiles / CUs) through the LDS request, so the
    // dispatcher spreads them over every CU instead of stacking two on some
    // while others idle.
    size_t launch_lds = lds_bytes;
    if (plan.path != RC_PATH_L2 && di->cus > 0 && di->lds_per_cu > 0) {
        const int64_t per = ((int64_t)p.ntiles + di->cus - 1) / di->cus;
        if (per >= 1 && per <= 3) {
            const size_t floor_bytes = di->lds_per_cu / (size_t)(per + 1) + 256;
            if (floor_bytes <= di->lds) launch_lds = std::max(launch_lds, floor_bytes);
        }
    }
    hipError_t e = launch_apply(p, plan, launch_lds, stream);
    return e == hipSuccess ? RC_OK : hip_fail(e);
}

}  // namespace
}  // namespace rc

using namespace rc;

extern "C" {

const char* rc_status_str(rc_status s) {
    switch (s) {
        case RC_OK: return "RC_OK";
        case RC_EINVAL: return "RC_EINVAL: invalid argument";
        case RC_ENOMEM: return "RC_ENOMEM: out of memory";
        case RC_EHIP: return "RC_EHIP: HIP runtime error";
        case RC_EBUSY: return "RC_EBUSY: busy";
        case RC_ECLOSED: return "RC_ECLOSED: closed";
    }
    return "rc_status: unknown";
}

int32_t rc_last_hip_error(void) { return t_last_hip; }

rc_status rc_lut_build(const double* coeffs, int32_t bands, int32_t detectors, int32_t levels,
                       uint16_t* lut, hipStream_t stream) {
    if (bands < 0 || detectors < 0) return RC_EINVAL;
    if (levels < RC_LEVELS_MIN || levels > RC_LEVELS_MAX) return RC_EINVAL;
    int64_t rows = 0, entries = 0, cbytes = 0, lbytes = 0;
    if (!mul_ok(bands, detectors, &rows) || !mul_ok(rows, levels, &entries) ||
        !mul_ok(entries, 2, &lbytes) || !mul_ok(rows, 32, &cbytes))
        return RC_EINVAL;
    if (rows == 0) return RC_OK;
    if (!coeffs || !lut) return RC_EINVAL;
    if (((uintptr_t)coeffs & 7u) || ((uintptr_t)lut & 1u)) return RC_EINVAL;
    if (overlaps(coeffs, (size_t)cbytes, lut, (size_t)lbytes)) return RC_EINVAL;
    int dev = 0;
    if (!current_device(&dev)) return RC_EHIP;
    hipError_t e = launch_lut_build(coeffs, rows, levels, lut, stream);
    return e == hipSuccess ? RC_OK : hip_fail(e);
}

rc_status rc_correct(const uint16_t* dn, const uint16_t* lut, int64_t lines, int32_t detectors,
                     int32_t bands, int32_t levels, uint16_t* out, hipStream_t stream) {
    return run_correct(dn, lut, lines, detectors, bands, levels, out, nullptr, stream);
}

rc_status rc_correct_plan(const uint16_t* dn, const uint16_t* lut, int64_t lines,
                          int32_t detectors, int32_t bands, int32_t levels, uint16_t* out,
                          const rc_plan* plan, hipStream_t stream) {
    if (!plan) return RC_EINVAL;
    return run_correct(dn, lut, lines, detectors, bands, levels, out, plan, stream);
}

size_t rc_correct_ws_bytes(int32_t detectors, int32_t bands, int32_t levels) {
    if (detectors <= 0 || bands <= 0 || !ws_path(levels)) return 0;
    return dense_ws_bytes(detectors, bands, levels);
}

rc_status rc_correct_ws(const uint16_t* dn, const uint16_t* lut, int64_t lines, int32_t detectors,
                        int32_t bands, int32_t levels, uint16_t* out, void* ws, size_t ws_bytes,
                        const rc_plan* plan, hipStream_t stream) {
    if (ws_path(levels) && detectors > 0 && bands > 0 && lines > 0 && !ws) return RC_EINVAL;
    return run_correct(dn, lut, lines, detectors, bands, levels, out, plan, stream, ws, ws_bytes);
}

rc_status rc_correct_pre(const uint16_t* dn, const uint16_t* lut, int64_t lines, int32_t detectors,
                         int32_t bands, int32_t levels, uint16_t* out, const void* ws,
                         size_t ws_bytes, const rc_plan* plan, hipStream_t stream) {
    if (!ws_path(levels)) return RC_EINVAL;
    if (detectors > 0 && bands > 0 && lines > 0 && !ws) return RC_EINVAL;
    return run_correct(dn, lut, lines, detectors, bands, levels, out, plan, stream,
                       const_cast<void*>(ws), ws_bytes, true);
}

rc_status rc_lut_build_ws(const double* coeffs, int32_t bands, int32_t detectors, int32_t levels,
                          uint16_t* lut, void* ws, size_t ws_bytes, hipStream_t stream) {
    if (bands < 0 || detectors < 0 || !ws_path(levels)) return RC_EINVAL;
    int64_t rows = 0, entries = 0, cbytes = 0, lbytes = 0;
    if (!mul_ok(bands, detectors, &rows) || !mul_ok(rows, levels, &entries) ||
        !mul_ok(entries, 2, &lbytes) || !mul_ok(rows, 32, &cbytes))
        return RC_EINVAL;
    if (rows == 0) return RC_OK;
    if (!coeffs || !lut || !ws) return RC_EINVAL;
    if (((uintptr_t)coeffs & 7u) || ((uintptr_t)lut & 1u) || ((uintptr_t)ws & 255u))
        return RC_EINVAL;
    const size_t need = dense_ws_bytes(detectors, bands, levels);
    if (ws_bytes < need) return RC_EINVAL;
    if (overlaps(coeffs, (size_t)cbytes, lut, (size_t)lbytes) ||
        overlaps(ws, need, coeffs, (size_t)cbytes) || overlaps(ws, need, lut, (size_t)lbytes))
        return RC_EINVAL;
    int dev = 0;
    if (!current_device(&dev)) return RC_EHIP;
    // The split run_correct uses: planes from byte 0, headers from the next
    // 256-byte boundary after them.
    const size_t n = (size_t)rows * (size_t)((levels + 63) / 64);
    uint64_t* planes = (uint64_t*)ws;
    int16_t* heads = (int16_t*)((char*)ws + ((n * 8 + 255) & ~(size_t)255));
    hipError_t e = launch_lut_build_ws(coeffs, rows, detectors, levels, lut, planes, heads, stream);
    return e == hipSuccess ? RC_OK : hip_fail(e);
}

rc_status rc_plan_for(int64_t lines, int32_t detectors, int32_t bands, int32_t levels,
                      const uint16_t* dn, const uint16_t* out, rc_plan* plan, int32_t* source) {
    if (!plan || lines <= 0 || detectors <= 0 || bands <= 0) return RC_EINVAL;
    if (levels < RC_LEVELS_MIN || levels > RC_LEVELS_MAX) return RC_EINVAL;
    const DeviceInfo* di = current_device();
    if (!di) return RC_EHIP;
    const int vmax = max_vec(dn, out, detectors, 8);
    const bool tuned = tuned_plan(lines, detectors, bands, levels, vmax, *di, plan);
    if (!tuned) default_plan(lines, detectors, bands, levels, vmax, *di, plan);
    if (source) *source = tuned ? 1 : 0;
    return RC_OK;
}

}  // extern "C"
