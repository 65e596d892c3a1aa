// Autotuner and plan cache for the correction kernel.
//
// rc_tune times candidate launch shapes (path, strip width, pixels per lane,
// workgroup size, unroll, line chunking, XCD remap, cache policy) on
// the caller's buffers with HIP events and keeps the fastest per shape
// class. Shape class = (arch, CU count, levels, ceil(log2 detectors),
// ceil(log2 lines), bands, largest usable vector width). Line chunking is
// stored as a chunk count, so one entry serves every line count of its
// class. The cache persists as one JSON object per line; rc_correct consults
// it (host only, no synchronisation) and falls back to the default plan.
// Batch entries ("kind":1, written by rc_batch_tune in batch.hip) hold the
// persistent batch kernel's tile shape for a class (levels, ceil(log2
// detectors), largest usable vector width); lines and bands are 0 there.
#include <dlfcn.h>
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "device_ops.h"
#include "kernels.h"
#include "rc.h"
#include "runtime.h"

namespace rc {

namespace {

struct Entry {
    std::string arch;
    int cus = 0;
    int levels = 0;
    int dclass = 0;
    int nclass = 0;
    int bands = 0;
    int vmax = 0;
    rc_plan plan{};
    int chunks = 1;  // line chunks per strip (chunk_lines = ceil(lines / chunks))
    double us = 0.0;
    int kind = 0;    // 0: plain-path plan, 1: batch tile shape
};

std::mutex g_mu;
std::vector<Entry> g_cache;
bool g_loaded = false;

int clog2(int64_t x) {
    int r = 0;
    while (((int64_t)1 << r) < x) ++r;
    return r;
}

std::string default_path() {
    const char* env = std::getenv("RC_TUNE_CACHE");
    if (env && *env) return env;
    Dl_info info;
    if (dladdr((void*)&default_path, &info) && info.dli_fname) {
        std::string p = info.dli_fname;
        const size_t slash = p.rfind('/');
        p = slash == std::string::npos ? std::string(".") : p.substr(0, slash);
        return p + "/tune_cache.json";
    }
    return "tune_cache.json";
}

// Minimal reader for the flat JSON objects written by save_locked().
// A number after "key": that converts to int32 exactly as written (the cache
// holds integers and one timing); anything else makes the line invalid.
bool get_num(const std::string& line, const char* key, double* out) {
    const std::string k = std::string("\"") + key + "\":";
    const size_t at = line.find(k);
    if (at == std::string::npos) return false;
    const char* begin = line.c_str() + at + k.size();
    char* end = nullptr;
    const double v = std::strtod(begin, &end);
    if (end == begin || !std::isfinite(v) || v < -2147483648.0 || v > 2147483647.0) return false;
    *out = v;
    return true;
}

bool get_str(const std::string& line, const char* key, std::string* out) {
    const std::string k = std::string("\"") + key + "\":";
    const size_t at = line.find(k);
    if (at == std::string::npos) return false;
    size_t begin = at + k.size();
    while (begin < line.size() && (line[begin] == ' ' || line[begin] == '\t')) ++begin;
    if (begin >= line.size() || line[begin] != '"') return false;
    ++begin;
    const size_t end = line.find('"', begin);
    if (end == std::string::npos) return false;
    *out = line.substr(begin, end - begin);
    return true;
}

bool parse_entry(const std::string& line, Entry* e) {
    double v[16];
    const char* keys[] = {"cus", "levels", "dclass", "nclass", "bands", "vmax", "path", "strip",
                          "vec", "threads", "unroll", "chunks", "xcd_remap", "nontemporal", "us"};
    for (int i = 0; i < 15; ++i)
        if (!get_num(line, keys[i], &v[i])) return false;
    if (!get_str(line, "arch", &e->arch)) return false;
    e->cus = (int)v[0];
    e->levels = (int)v[1];
    e->dclass = (int)v[2];
    e->nclass = (int)v[3];
    e->bands = (int)v[4];
    e->vmax = (int)v[5];
    e->plan.path = (int32_t)v[6];
    e->plan.strip = (int32_t)v[7];
    e->plan.vec = (int32_t)v[8];
    e->plan.threads = (int32_t)v[9];
    e->plan.unroll = (int32_t)v[10];
    e->chunks = std::max(1, (int)v[11]);
    e->plan.xcd_remap = (int32_t)v[12];
    e->plan.nontemporal = (int32_t)v[13];
    e->us = v[14];
    // Entries written before uneven strips existed have no "strips" key: 0.
    double st = 0.0;
    e->plan.strips = get_num(line, "strips", &st) ? (int32_t)st : 0;
    e->plan.lane_map = get_num(line, "lane_map", &st) ? (int32_t)st : 0;
    e->kind = get_num(line, "kind", &st) ? (int)st : 0;
    if (e->plan.strips < 0 || e->kind < 0 || e->kind > 1) return false;
    return true;
}

int load_locked(const std::string& path) {
    FILE* f = std::fopen(path.c_str(), "r");
    if (!f) return -1;
    std::vector<Entry> got;
    char buf[1024];
    while (std::fgets(buf, sizeof buf, f)) {
        Entry e;
        if (parse_entry(buf, &e)) got.push_back(e);
    }
    std::fclose(f);
    g_cache = got;
    return (int)got.size();
}

void ensure_loaded_locked() {
    if (g_loaded) return;
    g_loaded = true;
    load_locked(default_path());
}

int save_locked(const std::string& path) {
    const std::string tmp = path + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "w");
    if (!f) return -1;
    for (const Entry& e : g_cache) {
        std::fprintf(f,
                     "{\"arch\":\"%s\",\"cus\":%d,\"levels\":%d,\"dclass\":%d,\"nclass\":%d,"
                     "\"bands\":%d,\"vmax\":%d,\"path\":%d,\"strip\":%d,\"vec\":%d,"
                     "\"threads\":%d,\"unroll\":%d,\"chunks\":%d,\"xcd_remap\":%d,"
                     "\"nontemporal\":%d,\"strips\":%d,\"lane_map\":%d,\"kind\":%d,"
                     "\"us\":%.3f}\n",
                     e.arch.c_str(), e.cus, e.levels, e.dclass, e.nclass, e.bands, e.vmax,
                     e.plan.path, e.plan.strip, e.plan.vec, e.plan.threads, e.plan.unroll,
                     e.chunks, e.plan.xcd_remap, e.plan.nontemporal, e.plan.strips,
                     e.plan.lane_map, e.kind, e.us);
    }
    const bool ok = std::fclose(f) == 0;
    if (!ok || std::rename(tmp.c_str(), path.c_str()) != 0) return -1;
    return (int)g_cache.size();
}

Entry key_of(int64_t lines, int32_t detectors, int32_t bands, int32_t levels, int vmax,
             const DeviceInfo& di) {
    Entry k;
    k.arch = di.arch;
    k.cus = di.cus;
    k.levels = levels;
    k.dclass = clog2(detectors);
    k.nclass = clog2(lines);
    k.bands = bands;
    k.vmax = vmax;
    return k;
}

bool same_class(const Entry& a, const Entry& b) {
    return a.kind == b.kind && a.arch == b.arch && a.cus == b.cus && a.levels == b.levels &&
           a.dclass == b.dclass && a.nclass == b.nclass && a.bands == b.bands && a.vmax == b.vmax;
}

Entry batch_key(int32_t detectors, int32_t levels, int vmax, const DeviceInfo& di) {
    Entry k = key_of(0, detectors, 0, levels, vmax, di);
    k.kind = 1;
    return k;
}

int chunk_count(int64_t lines, int32_t chunk_lines) {
    return (int)std::min<int64_t>(INT32_MAX, (lines + chunk_lines - 1) / chunk_lines);
}

}  // namespace

bool tuned_plan(int64_t lines, int32_t detectors, int32_t bands, int32_t levels, int vmax,
                const DeviceInfo& di, rc_plan* plan) {
    const Entry k = key_of(lines, detectors, bands, levels, vmax, di);
    rc_plan found;
    int chunks = 1;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        ensure_loaded_locked();
        auto it = std::find_if(g_cache.begin(), g_cache.end(),
                               [&](const Entry& e) { return same_class(e, k); });
        if (it == g_cache.end()) return false;
        found = it->plan;
        chunks = it->chunks;
    }
    found.chunk_lines = (int32_t)std::max<int64_t>(1, (lines + chunks - 1) / chunks);
    ApplyParams p{};
    size_t lds = 0;
    if (check_plan(found, lines, detectors, bands, levels, vmax, di, &p, &lds) != RC_OK)
        return false;
    *plan = found;
    return true;
}

bool tuned_batch_shape(int32_t detectors, int32_t levels, int vmax, const DeviceInfo& di,
                       rc_plan* plan) {
    const Entry k = batch_key(detectors, levels, vmax, di);
    std::lock_guard<std::mutex> lk(g_mu);
    ensure_loaded_locked();
    auto it = std::find_if(g_cache.begin(), g_cache.end(),
                           [&](const Entry& e) { return same_class(e, k); });
    if (it == g_cache.end()) return false;
    *plan = it->plan;
    return true;
}

void store_batch_shape(int32_t detectors, int32_t levels, int vmax, const DeviceInfo& di,
                       const rc_plan& plan, double us) {
    Entry ent = batch_key(detectors, levels, vmax, di);
    ent.plan = plan;
    ent.us = us;
    std::lock_guard<std::mutex> lk(g_mu);
    ensure_loaded_locked();
    auto it = std::find_if(g_cache.begin(), g_cache.end(),
                           [&](const Entry& x) { return same_class(x, ent); });
    if (it != g_cache.end()) *it = ent;
    else g_cache.push_back(ent);
}

namespace {

std::vector<rc_plan> candidates(int64_t lines, int32_t detectors, int32_t bands, int32_t levels,
                                int vmax, const DeviceInfo& di, int effort) {
    (void)bands;
    std::vector<rc_plan> out;
    rc_plan def;
    default_plan(lines, detectors, bands, levels, vmax, di, &def);
    out.push_back(def);
    const int64_t dcap = (int64_t)1 << clog2(std::max(detectors, 1));
    auto add = [&](int path, int W, int vec, int threads, int unroll, int nt, int k) {
        if (k > lines || W / vec > threads || W < vec || vec > vmax) return;
        rc_plan p;
        std::memset(&p, 0, sizeof p);
        p.path = path;
        p.strip = W;
        p.vec = vec;
        p.threads = threads;
        p.unroll = unroll;
        p.xcd_remap = 1;
        p.nontemporal = nt;
        p.chunk_lines = (int32_t)((lines + k - 1) / k);
        out.push_back(p);
    };
    // Balanced tilings: one tile per resident workgroup (1 or 2 per CU), or
    // two rounds of them; pixels per lane up to 8 (16-byte accesses).
    {
        std::vector<int> vecs8;
        for (int v = std::min(vmax, 8); v >= 1 && vecs8.size() < (effort ? 3u : 2u); v >>= 1)
            vecs8.push_back(v);
        const int cus = std::max(1, di.cus);
        for (int path : {RC_PATH_PACKED, RC_PATH_LDS})
            for (int per_cu : {1, 2}) {
                const size_t budget =
                    std::min(di.lds, (di.lds_per_cu ? di.lds_per_cu : di.lds) / per_cu);
                const int wmax = widest_strip(path, levels, budget);
                if (wmax < 16) continue;
                for (int threads : {256, 512, 1024}) {
                    if (threads * per_cu > 2048) continue;
                    for (int vec : vecs8)
                        for (int unroll : {4, 8})
                            for (int nt : {0, 2})
                                for (int rounds : {1, 2})
                                    for (int lane_map : {0, 1}) {
                                        if (vec == 8 && unroll != 4) continue;
                                        rc_plan p;
                                        std::memset(&p, 0, sizeof p);
                                        p.path = path;
                                        p.vec = vec;
                                        p.threads = threads;
                                        p.unroll = unroll;
                                        p.xcd_remap = 1;
                                        p.nontemporal = nt;
                                        p.lane_map = lane_map;
                                        if (!balanced_tiling(lines, detectors, bands, vec, wmax,
                                                             (int64_t)per_cu * cus * rounds,
                                                             threads, unroll, &p.strips, &p.strip,
                                                             &p.chunk_lines))
                                            continue;
                                        if (p.strip / vec > threads) continue;
                                        out.push_back(p);
                                    }
                }
            }
    }
    std::vector<int> vecs;
    if (vmax >= 8) vecs.push_back(8);
    if (vmax >= 4) vecs.push_back(4);
    if (vmax >= 2) vecs.push_back(2);
    if (effort > 0 || vmax == 1) vecs.push_back(1);
    if (effort == 0 && vecs.size() > 2) vecs.resize(2);
    const std::vector<int> threads_l = effort ? std::vector<int>{256, 512, 1024}
                                              : std::vector<int>{512, 1024};
    const std::vector<int> unrolls = effort ? std::vector<int>{4, 8, 16} : std::vector<int>{4, 8};
    const std::vector<int> ks = effort ? std::vector<int>{1, 2, 3, 4, 6, 8, 12}
                                       : std::vector<int>{1, 2, 4};
    // LDS paths: the two widest strips that fit (the measured throughput of
    // strip-shaped streams grows with the strip width).
    for (int path : {RC_PATH_PACKED, RC_PATH_LDS, RC_PATH_DENSE}) {
        if (path == RC_PATH_DENSE && levels > kDenseMaxLevels) continue;
        std::vector<int> widths;
        for (int W = 256; W >= 8 && widths.size() < 2; W >>= 1) {
            if (plan_lds_bytes(path, W, levels) > di.lds) continue;
            if (W > std::max<int64_t>(dcap, 8)) continue;
            widths.push_back(W);
        }
        for (int W : widths)
            for (int vec : vecs)
                for (int threads : threads_l)
                    for (int unroll : unrolls)
                        for (int nt = 0; nt < (effort ? kPolicies : 3); ++nt)
                            for (int k : ks) {
                                if (vec == 8 && unroll != 4) continue;
                                if (path == RC_PATH_DENSE && threads > kDenseMaxThreads) continue;
                                add(path, W, vec, threads, unroll, nt, k);
                            }
    }
    // The L2 path: a few shapes, line chunks sized so an XCD's CUs share a strip.
    for (int W : {32, 64, 128})
        for (int vec : vecs)
            for (int k : {32, 64}) add(RC_PATH_L2, W, vec, 256, 8, 0, k);
    return out;
}

}  // namespace
}  // namespace rc

using namespace rc;

extern "C" {

rc_status rc_tune(const uint16_t* dn, const uint16_t* lut, int64_t lines, int32_t detectors,
                  int32_t bands, int32_t levels, uint16_t* out, int32_t effort, rc_plan* best,
                  float* best_us, hipStream_t stream) {
    if (lines <= 0 || detectors <= 0 || bands <= 0) return RC_EINVAL;
    if (levels < RC_LEVELS_MIN || levels > RC_LEVELS_MAX) return RC_EINVAL;
    if (!dn || !lut || !out || dn == out) return RC_EINVAL;
    const DeviceInfo* di = current_device();
    if (!di) return RC_EHIP;
    const int vmax = max_vec(dn, out, detectors, 8);
    std::vector<rc_plan> cands = candidates(lines, detectors, bands, levels, vmax, *di, effort);
    hipEvent_t e0, e1;
    hipError_t e = hipEventCreate(&e0);
    if (e != hipSuccess) return hip_fail(e);
    e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_fail(e);
    }
    // Back-to-back calls on one set of buffers rank plans on warm caches. That
    // is what a large shape sees anyway, but a shape whose image and LUT fit
    // the caches (L2 and the 256 MB MALL) would be ranked on data a stream of
    // different scenes never has cached. For those, each timed call follows a
    // write of kEvict scratch bytes that evicts everything and a copy of the
    // LUT that brings it back, as rc_lut_build leaves it just before
    // rc_correct; the scratch is allocated for the duration of this call.
    const size_t lut_bytes = (size_t)bands * (size_t)detectors * (size_t)levels * 2;
    const double footprint = 4.0 * (double)lines * detectors * bands + (double)lut_bytes;
    const size_t kEvict = (size_t)512 << 20;
    void* scratch = nullptr;
    const bool cold = footprint < (double)kEvict &&
                      hipMalloc(&scratch, kEvict + lut_bytes) == hipSuccess;
    const int reps = cold ? 5 : 3;
    float best_t = 1e30f;
    rc_plan best_p = cands[0];
    rc_status st = RC_OK;
    for (const rc_plan& p : cands) {
        if (rc_correct_plan(dn, lut, lines, detectors, bands, levels, out, &p, stream) != RC_OK)
            continue;  // not runnable for this shape/device
        float t = 0.f;
        if (cold) {
            for (int r = 0; r < reps && e == hipSuccess; ++r) {
                float one = 0.f;
                if ((e = hipMemsetAsync(scratch, r & 0xff, kEvict, stream)) != hipSuccess) break;
                if ((e = hipMemcpyAsync((char*)scratch + kEvict, lut, lut_bytes,
                                        hipMemcpyDeviceToDevice, stream)) != hipSuccess)
                    break;
                if ((e = hipEventRecord(e0, stream)) != hipSuccess) break;
                rc_correct_plan(dn, lut, lines, detectors, bands, levels, out, &p, stream);
                if ((e = hipEventRecord(e1, stream)) != hipSuccess) break;
                if ((e = hipEventSynchronize(e1)) != hipSuccess) break;
                if ((e = hipEventElapsedTime(&one, e0, e1)) != hipSuccess) break;
                t += one;
            }
            if (e != hipSuccess) break;
        } else {
            if ((e = hipEventRecord(e0, stream)) != hipSuccess) break;
            for (int r = 0; r < reps; ++r)
                rc_correct_plan(dn, lut, lines, detectors, bands, levels, out, &p, stream);
            if ((e = hipEventRecord(e1, stream)) != hipSuccess) break;
            if ((e = hipEventSynchronize(e1)) != hipSuccess) break;
            if ((e = hipEventElapsedTime(&t, e0, e1)) != hipSuccess) break;
        }
        t *= 1000.f / reps;
        if (t < best_t) {
            best_t = t;
            best_p = p;
        }
    }
    if (e != hipSuccess) st = hip_fail(e);
    if (scratch) {
        // Nothing may still read or write the scratch when it is freed.
        const hipError_t se = hipStreamSynchronize(stream);
        if (se != hipSuccess && st == RC_OK) st = hip_fail(se);
        (void)hipFree(scratch);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != RC_OK) return st;
    if (best) *best = best_p;
    if (best_us) *best_us = best_t;
    Entry ent = key_of(lines, detectors, bands, levels, vmax, *di);
    ent.plan = best_p;
    ent.chunks = chunk_count(lines, best_p.chunk_lines);
    ent.us = best_t;
    std::lock_guard<std::mutex> lk(g_mu);
    ensure_loaded_locked();
    auto it = std::find_if(g_cache.begin(), g_cache.end(),
                           [&](const Entry& x) { return same_class(x, ent); });
    if (it != g_cache.end()) *it = ent;
    else g_cache.push_back(ent);
    return RC_OK;
}

int32_t rc_tune_save(const char* path) {
    std::lock_guard<std::mutex> lk(g_mu);
    ensure_loaded_locked();
    return save_locked(path && *path ? path : default_path());
}

int32_t rc_tune_load(const char* path) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_loaded = true;
    const int n = load_locked(path && *path ? path : default_path());
    if (n < 0) g_cache.clear();
    return n;
}

void rc_tune_clear(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_loaded = true;
    g_cache.clear();
}

int32_t rc_tune_count(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    ensure_loaded_locked();
    return (int32_t)g_cache.size();
}

}  // extern "C"
