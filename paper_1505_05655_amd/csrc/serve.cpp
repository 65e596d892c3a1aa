// Serving runtime: continuous batching of correction jobs.
//
// The paper's framework (§II) has clients submit a task together with its
// data to a GPU server and get the results back. Here the server is an
// in-process runtime: rc_server_submit hands over a job (host buffers), a
// scheduler thread admits it when its bytes fit a device-memory arena and a
// job slot is free, copies it in piece by piece (a piece = one band's run of
// lines) on a host-to-device stream, and feeds the tiles of every piece that
// has arrived, from all admitted jobs, into quanta of the persistent fused
// kernel on the compute stream. When the last tile of a piece has been
// issued, the piece is copied back on a device-to-host stream behind that
// quantum. When the output buffer is pinned host memory that the device can
// address (rc_host_alloc), the kernel writes the corrected lines straight to
// it instead: the copy back would otherwise run as a copy kernel competing
// with the quanta for the CUs. Copies and kernels overlap, and a job arriving
// while others run joins the next quantum.
//
// Every kernel launched here terminates on its own (no kernel waits on host
// memory); the scheduler polls HIP events from the host.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "batch.h"
#include "device_ops.h"
#include "kernels.h"
#include "rc.h"
#include "runtime.h"

namespace rc {
namespace {

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// First-fit allocator over the server's device arena (host bookkeeping).
class Arena {
public:
    void init(size_t bytes) {
        free_.clear();
        if (bytes) free_[0] = bytes;
        total_ = bytes;
        used_ = 0;
    }
    bool alloc(size_t bytes, size_t* off) {
        bytes = round_up(std::max<size_t>(bytes, 1), 256);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes, start = it->first + bytes;
            free_.erase(it);
            if (rest) free_[start] = rest;
            used_ += bytes;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = round_up(std::max<size_t>(bytes, 1), 256);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t total() const { return total_; }
    size_t used() const { return used_; }

private:
    std::map<size_t, size_t> free_;
    size_t total_ = 0, used_ = 0;
};

enum PieceState { kLoading = 0, kReady = 1, kIssued = 2, kDone = 3 };

struct Piece {
    int32_t band = 0;
    int64_t n0 = 0, n1 = 0;
    int32_t next_tile = 0;  // next strip to issue
    int32_t ntiles = 0;
    int state = kLoading;
    hipEvent_t ev_in = nullptr;   // recorded after its host-to-device copy
    hipEvent_t ev_out = nullptr;  // recorded after its device-to-host copy
};

struct Job {
    uint64_t id = 0;
    rc_host_job host{};
    int64_t pixels = 0, rows = 0, lut_n = 0;
    size_t off = 0, bytes = 0;  // arena region
    size_t off_coeffs = 0, off_lut = 0, off_dn = 0, off_out = 0;
    uint16_t* direct_out = nullptr;  // device address of the pinned host output, or null
    BatchReq req{};             // device pointers filled at admission
    std::vector<Piece> pieces;
    size_t next_arrival = 0;    // first piece not yet seen arrived
    int pieces_open = 0;        // pieces whose copy back has not completed
    bool built = false;         // global LUT build enqueued (L2-path jobs)
    hipEvent_t ev_coeffs = nullptr;  // recorded after the coefficient copy
    hipEvent_t ev_lut = nullptr;
    bool lut_enqueued = false;
    int status = RC_OK;
    bool done = false;
    double submit_s = 0, admit_s = 0, start_s = 0, done_s = 0;
};

// One descriptor slot of the quantum ring. The descriptors live in pinned
// host memory that the kernel reads directly (a quantum's few KB would
// otherwise be a DMA copy queued behind the bulk piece copies).
struct Slot {
    unsigned int* d_counters = nullptr;
    BatchReq* h_reqs = nullptr;    // pinned, written by the scheduler
    BatchTile* h_tiles = nullptr;  // pinned, written by the scheduler
    const BatchReq* k_reqs = nullptr;    // the same memory, as the device sees it
    const BatchTile* k_tiles = nullptr;
    hipEvent_t ev = nullptr;
    bool busy = false;
};

constexpr int kSlots = 4;
constexpr int kInFlight = 2;

}  // namespace
}  // namespace rc

using namespace rc;

struct rc_server {
    int device = 0;
    rc_server_opts opts{};
    const DeviceInfo* di = nullptr;
    size_t lds = 0;
    int grid = 0;
    unsigned char* arena_base = nullptr;
    Arena arena;
    hipStream_t s_in = nullptr, s_comp = nullptr, s_out = nullptr;
    Slot slots[kSlots];
    std::vector<hipEvent_t> event_pool;

    std::mutex mu;
    std::condition_variable cv_work;  // scheduler wake-up
    std::condition_variable cv_done;  // waiters
    std::deque<std::shared_ptr<Job>> pending;
    std::vector<std::shared_ptr<Job>> active;  // admitted, in admission order
    std::unordered_map<uint64_t, std::shared_ptr<Job>> jobs;
    uint64_t next_id = 1;
    bool stop = false;
    int waiters = 0;  // threads inside rc_server_wait
    int failed = 0;   // hipError_t that stopped the server
    rc_server_stats stats{};
    std::thread thread;
};

namespace {

hipEvent_t get_event(rc_server* s) {
    if (!s->event_pool.empty()) {
        hipEvent_t e = s->event_pool.back();
        s->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    return e;
}

void put_event(rc_server* s, hipEvent_t& e) {
    if (e) s->event_pool.push_back(e);
    e = nullptr;
}

// Device bytes a job occupies: coefficients, LUT, input image and, unless the
// kernel writes the host output directly, the output image.
size_t job_bytes(const rc_host_job& j, bool direct_out, size_t* off_lut, size_t* off_dn,
                 size_t* off_out) {
    const size_t rows = (size_t)j.bands * (size_t)j.detectors;
    const size_t px = rows * (size_t)j.lines;
    size_t o = round_up(rows * 32, 256);
    *off_lut = o;
    o += round_up(rows * (size_t)j.levels * 2, 256);
    *off_dn = o;
    o += round_up(px * 2, 256);
    *off_out = o;
    if (!direct_out) o += round_up(px * 2, 256);
    return o;
}

// Device address of [p, p + bytes) if it is one pinned host allocation the
// device maps contiguously, else null (HIP's error state is cleared).
uint16_t* mapped_host(const void* p, size_t bytes) {
    void* d0 = nullptr;
    void* d1 = nullptr;
    const char* last = (const char*)p + (bytes - 1);
    if (!p || bytes == 0 || hipHostGetDevicePointer(&d0, const_cast<void*>(p), 0) != hipSuccess ||
        hipHostGetDevicePointer(&d1, (void*)last, 0) != hipSuccess || !d0 ||
        (const char*)d1 - (const char*)d0 != (ptrdiff_t)(bytes - 1)) {
        (void)hipGetLastError();
        return nullptr;
    }
    return (uint16_t*)d0;
}

rc_status validate_job(const rc_host_job& j) {
    if (j.lines < 0 || j.detectors < 0 || j.bands < 0 || j.reserved != 0) return RC_EINVAL;
    if (j.levels < RC_LEVELS_MIN || j.levels > RC_LEVELS_MAX) return RC_EINVAL;
    int64_t rows = 0, px = 0, lut_n = 0;
    if (!mul_ok(j.bands, j.detectors, &rows) || !mul_ok(rows, j.lines, &px) ||
        !mul_ok(rows, j.levels, &lut_n) || px > INT64_MAX / 4 || lut_n > INT64_MAX / 4)
        return RC_EINVAL;
    if (rows > 0 && !j.coeffs) return RC_EINVAL;
    if (px > 0 && (!j.dn || !j.out)) return RC_EINVAL;
    if (max_chunk_lines(std::max(j.detectors, 1), kBatchThreads, kBatchUnroll) < 1)
        return RC_EINVAL;
    return RC_OK;
}

// Marks the server failed: every unfinished job completes with RC_EHIP.
void fail_all(rc_server* s, hipError_t e) {
    s->failed = (int)e;
    // Copies and quanta already enqueued for the active jobs may still read
    // or write their host buffers (pinned staging, or out directly): all
    // three streams drain before any job is reported finished, so that a
    // caller may free its buffers as soon as wait/poll returns. After a
    // device fault these waits return at once, with the error.
    (void)hipStreamSynchronize(s->s_in);
    (void)hipStreamSynchronize(s->s_comp);
    (void)hipStreamSynchronize(s->s_out);
    const double t = now_s();
    for (auto& j : s->active) {
        j->status = RC_EHIP;
        j->done = true;
        j->done_s = t;
    }
    s->active.clear();
    for (auto& j : s->pending) {
        j->status = RC_EHIP;
        j->done = true;
        j->done_s = t;
    }
    s->pending.clear();
    s->cv_done.notify_all();
}

// Admission: arena region, plan, pieces, and the copies in.
hipError_t admit(rc_server* s, const std::shared_ptr<Job>& jp) {
    Job& j = *jp;
    const rc_host_job& h = j.host;
    unsigned char* base = s->arena_base + j.off;
    j.off_coeffs = 0;
    job_bytes(h, j.direct_out != nullptr, &j.off_lut, &j.off_dn, &j.off_out);
    BatchReq& q = j.req;
    std::memset(&q, 0, sizeof q);
    q.coeffs = (const double*)(base + j.off_coeffs);
    q.lut = (uint16_t*)(base + j.off_lut);
    q.dn = (const uint16_t*)(base + j.off_dn);
    q.out = j.direct_out ? j.direct_out : (uint16_t*)(base + j.off_out);
    q.lines = h.lines;
    q.detectors = h.detectors;
    q.bands = h.bands;
    q.levels = h.levels;
    q.lut_vec = h.levels % 8 == 0 ? 1 : 0;  // arena offsets are 256-byte aligned
    if (j.rows > 0) {
        const int vmax = j.pixels > 0 ? max_vec(q.dn, q.out, h.detectors) : 1;
        const int64_t lines_p = std::max<int64_t>(h.lines, 1);
        rc_plan p;
        if (!tuned_plan(lines_p, h.detectors, h.bands, h.levels, vmax, *s->di, &p))
            pow2_plan(lines_p, h.detectors, h.bands, h.levels, vmax, *s->di, &p);
        fit_request_plan(p, h.levels, s->lds, false, &q);
    }
    // Pieces: per band, runs of lines of about piece_pixels pixels.
    const int64_t cap = std::min<int64_t>(
        8192, max_chunk_lines(std::max(h.detectors, 1), kBatchThreads, kBatchUnroll));
    int64_t per = std::max<int64_t>(1, s->opts.piece_pixels / std::max(h.detectors, 1));
    per = std::min(per, cap);
    const int W = 1 << q.log_strip;
    const int32_t strips = h.detectors > 0 ? (h.detectors + W - 1) / W : 0;
    if (j.rows > 0) {
        for (int32_t b = 0; b < h.bands; ++b) {
            if (h.lines == 0) {
                if (!q.fused) continue;  // the build kernel alone produces the LUT
                Piece pc;
                pc.band = b;
                pc.ntiles = strips;
                j.pieces.push_back(pc);
                continue;
            }
            for (int64_t n0 = 0; n0 < h.lines; n0 += per) {
                Piece pc;
                pc.band = b;
                pc.n0 = n0;
                pc.n1 = std::min(h.lines, n0 + per);
                pc.ntiles = strips;
                j.pieces.push_back(pc);
            }
        }
    }
    // Copies in: coefficients first, then each piece (events in order).
    hipError_t e = hipSuccess;
    if (j.rows > 0) {
        e = hipMemcpyAsync((void*)q.coeffs, h.coeffs, (size_t)j.rows * 32, hipMemcpyHostToDevice,
                           s->s_in);
        if (e != hipSuccess) return e;
    }
    j.ev_coeffs = get_event(s);
    if (!j.ev_coeffs) return hipErrorOutOfMemory;
    if ((e = hipEventRecord(j.ev_coeffs, s->s_in)) != hipSuccess) return e;
    for (Piece& pc : j.pieces) {
        if (pc.n1 > pc.n0) {
            const size_t first = ((size_t)pc.band * (size_t)h.lines + (size_t)pc.n0) *
                                 (size_t)h.detectors;
            const size_t n = (size_t)(pc.n1 - pc.n0) * (size_t)h.detectors;
            e = hipMemcpyAsync((void*)(q.dn + first), h.dn + first, n * 2, hipMemcpyHostToDevice,
                               s->s_in);
            if (e != hipSuccess) return e;
        }
        pc.ev_in = get_event(s);
        if (!pc.ev_in) return hipErrorOutOfMemory;
        if ((e = hipEventRecord(pc.ev_in, s->s_in)) != hipSuccess) return e;
    }
    j.pieces_open = (int)j.pieces.size();
    j.admit_s = now_s();
    return hipSuccess;
}

// Enqueues the copy back of a piece behind the quantum event `after`. With a
// direct output the piece is done when the quantum is: its event is recorded
// on the compute stream right behind it.
hipError_t finish_piece(rc_server* s, Job& j, Piece& pc, hipEvent_t after) {
    const rc_host_job& h = j.host;
    if (j.direct_out) {
        pc.ev_out = get_event(s);
        if (!pc.ev_out) return hipErrorOutOfMemory;
        pc.state = kIssued;
        return hipEventRecord(pc.ev_out, s->s_comp);
    }
    hipError_t e = hipStreamWaitEvent(s->s_out, after, 0);
    if (e != hipSuccess) return e;
    if (pc.n1 > pc.n0) {
        const size_t first =
            ((size_t)pc.band * (size_t)h.lines + (size_t)pc.n0) * (size_t)h.detectors;
        const size_t n = (size_t)(pc.n1 - pc.n0) * (size_t)h.detectors;
        e = hipMemcpyAsync(h.out + first, j.req.out + first, n * 2, hipMemcpyDeviceToHost,
                           s->s_out);
        if (e != hipSuccess) return e;
    }
    pc.ev_out = get_event(s);
    if (!pc.ev_out) return hipErrorOutOfMemory;
    pc.state = kIssued;
    return hipEventRecord(pc.ev_out, s->s_out);
}

// The LUT copy back (if the client asked for it), behind `after`.
hipError_t copy_lut(rc_server* s, Job& j, hipEvent_t after) {
    hipError_t e = hipSuccess;
    if (after && (e = hipStreamWaitEvent(s->s_out, after, 0)) != hipSuccess) return e;
    if (j.host.lut && j.lut_n > 0) {
        e = hipMemcpyAsync(j.host.lut, j.req.lut, (size_t)j.lut_n * 2, hipMemcpyDeviceToHost,
                           s->s_out);
        if (e != hipSuccess) return e;
    }
    j.ev_lut = get_event(s);
    if (!j.ev_lut) return hipErrorOutOfMemory;
    j.lut_enqueued = true;
    return hipEventRecord(j.ev_lut, s->s_out);
}

// Builds and launches one quantum from the ready pieces (round-robin over
// pieces in admission order). Returns false when there was nothing to issue
// or no free slot.
bool launch_quantum(rc_server* s, hipError_t* err) {
    *err = hipSuccess;
    int slot = -1;
    int busy = 0;
    for (int k = 0; k < kSlots; ++k) {
        if (s->slots[k].busy) ++busy;
        else if (slot < 0) slot = k;
    }
    if (slot < 0 || busy >= kInFlight) return false;
    // Tiles of an L2-path job are issued only after its LUT build was
    // enqueued on the compute stream (stream order then covers it).
    std::vector<std::pair<Job*, Piece*>> ready;
    for (auto& jp : s->active) {
        if (!jp->req.fused && !jp->built) continue;
        for (Piece& pc : jp->pieces)
            if (pc.state == kReady && pc.next_tile < pc.ntiles) ready.push_back({jp.get(), &pc});
    }
    if (ready.empty()) return false;
    Slot& sl = s->slots[slot];
    const int max_tiles = s->opts.max_quantum_tiles;
    const int per_piece = std::max(1, max_tiles / (int)ready.size());
    int nt = 0, nreq = 0;
    std::unordered_map<Job*, int> req_index;
    std::vector<std::pair<Job*, Piece*>> completed;
    for (auto& rp : ready) {
        Job* j = rp.first;
        Piece* pc = rp.second;
        if (nt >= max_tiles) break;
        auto it = req_index.find(j);
        int ri;
        if (it == req_index.end()) {
            if (nreq >= s->opts.max_jobs) continue;
            ri = nreq++;
            req_index[j] = ri;
            sl.h_reqs[ri] = j->req;
        } else {
            ri = it->second;
        }
        const int W = 1 << j->req.log_strip;
        const int take = std::min(per_piece, std::min(pc->ntiles - pc->next_tile, max_tiles - nt));
        for (int k = 0; k < take; ++k) {
            BatchTile& tl = sl.h_tiles[nt++];
            tl.req = ri;
            tl.band = pc->band;
            tl.d0 = (pc->next_tile + k) * W;
            tl.pad = 0;
            tl.n0 = pc->n0;
            tl.n1 = pc->n1;
        }
        pc->next_tile += take;
        if (j->start_s == 0) j->start_s = now_s();
        if (pc->next_tile == pc->ntiles) completed.push_back(rp);
    }
    if (nt == 0) return false;
    hipError_t e;
    // The host stores above are complete before the launch is submitted.
    std::atomic_thread_fence(std::memory_order_seq_cst);
    if ((e = launch_batch_apply(sl.k_reqs, sl.k_tiles, single_queue(nt), sl.d_counters,
                                std::min(s->grid, nt), s->lds, s->s_comp)) != hipSuccess ||
        (e = hipEventRecord(sl.ev, s->s_comp)) != hipSuccess) {
        *err = e;
        return false;
    }
    sl.busy = true;
    s->stats.quanta += 1;
    s->stats.tiles += (uint64_t)nt;
    for (auto& rp : completed) {
        if ((e = finish_piece(s, *rp.first, *rp.second, sl.ev)) != hipSuccess) {
            *err = e;
            return false;
        }
        // Last piece of the job issued: queue the LUT copy behind this quantum.
        Job& j = *rp.first;
        bool all = true;
        for (Piece& pc : j.pieces) all &= pc.state != kLoading && pc.state != kReady;
        if (all && !j.lut_enqueued && (e = copy_lut(s, j, sl.ev)) != hipSuccess) {
            *err = e;
            return false;
        }
    }
    return true;
}

void scheduler(rc_server* s) {
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        bool progress = false;
        hipError_t e = hipSuccess;
        // Admission in arrival order while memory and job slots allow.
        while (!s->failed && !s->stop && !s->pending.empty() &&
               (int)s->active.size() < s->opts.max_jobs) {
            auto jp = s->pending.front();
            if (!s->arena.alloc(jp->bytes, &jp->off)) break;
            s->pending.pop_front();
            s->active.push_back(jp);
            if ((e = admit(s, jp)) != hipSuccess) break;
            progress = true;
        }
        if (e != hipSuccess) {
            fail_all(s, e);
            continue;
        }
        // Arrivals of pieces (in copy order per job).
        for (auto& jp : s->active) {
            Job& j = *jp;
            while (j.next_arrival < j.pieces.size()) {
                Piece& pc = j.pieces[j.next_arrival];
                const hipError_t q = hipEventQuery(pc.ev_in);
                if (q == hipErrorNotReady) break;
                if (q != hipSuccess) {
                    e = q;
                    break;
                }
                put_event(s, pc.ev_in);
                pc.state = kReady;
                ++j.next_arrival;
                progress = true;
            }
            if (e != hipSuccess) break;
            // L2-path jobs: build the global LUT once the coefficients are in.
            if (!j.built && !j.req.fused && j.rows > 0) {
                const hipError_t q = hipEventQuery(j.ev_coeffs);
                if (q == hipSuccess) {
                    if ((e = launch_lut_build(j.req.coeffs, j.rows, j.host.levels, j.req.lut,
                                              s->s_comp)) != hipSuccess)
                        break;
                    j.built = true;
                    progress = true;
                } else if (q != hipErrorNotReady) {
                    e = q;
                    break;
                }
            }
            // Jobs without pieces (LUT only, or empty): queue the LUT copy
            // back once the LUT exists.
            if (j.pieces.empty() && !j.lut_enqueued && (j.built || j.rows == 0)) {
                hipEvent_t ev = get_event(s);
                if (!ev) {
                    e = hipErrorOutOfMemory;
                    break;
                }
                if ((e = hipEventRecord(ev, s->s_comp)) != hipSuccess) break;
                e = copy_lut(s, j, ev);
                put_event(s, ev);
                if (e != hipSuccess) break;
                progress = true;
            }
        }
        if (e != hipSuccess) {
            fail_all(s, e);
            continue;
        }
        // Quanta: free finished slots, then issue while work and slots remain.
        for (Slot& sl : s->slots) {
            if (!sl.busy) continue;
            const hipError_t q = hipEventQuery(sl.ev);
            if (q == hipSuccess) {
                sl.busy = false;
                progress = true;
            } else if (q != hipErrorNotReady) {
                e = q;
            }
        }
        while (e == hipSuccess && launch_quantum(s, &e)) progress = true;
        if (e != hipSuccess) {
            fail_all(s, e);
            continue;
        }
        // Completions: every piece copied back and the LUT copy done.
        for (size_t k = 0; k < s->active.size();) {
            Job& j = *s->active[k];
            for (Piece& pc : j.pieces) {
                if (pc.state != kIssued) continue;
                const hipError_t q = hipEventQuery(pc.ev_out);
                if (q == hipErrorNotReady) continue;
                if (q != hipSuccess) {
                    e = q;
                    break;
                }
                put_event(s, pc.ev_out);
                pc.state = kDone;
                --j.pieces_open;
                progress = true;
            }
            if (e != hipSuccess) break;
            bool finished = j.pieces_open == 0 && j.lut_enqueued;
            if (finished) {
                const hipError_t q = hipEventQuery(j.ev_lut);
                if (q == hipErrorNotReady) finished = false;
                else if (q != hipSuccess) {
                    e = q;
                    break;
                }
            }
            if (finished) {
                put_event(s, j.ev_lut);
                put_event(s, j.ev_coeffs);
                s->arena.release(j.off, j.bytes);
                j.done = true;
                j.done_s = now_s();
                j.status = RC_OK;
                s->stats.completed += 1;
                s->stats.pixels += (uint64_t)j.pixels;
                s->active.erase(s->active.begin() + (long)k);
                s->cv_done.notify_all();
                progress = true;
                continue;
            }
            ++k;
        }
        if (e != hipSuccess) {
            fail_all(s, e);
            continue;
        }
        if (s->stop && s->active.empty()) {
            // Jobs never admitted are refused.
            for (auto& jp : s->pending) {
                jp->status = RC_ECLOSED;
                jp->done = true;
                jp->done_s = now_s();
            }
            s->pending.clear();
            s->cv_done.notify_all();
            break;
        }
        if (!progress) {
            if (s->active.empty() && (s->pending.empty() || s->failed)) {
                s->cv_work.wait(lk);  // nothing in flight: sleep until a submit or stop
            } else {
                lk.unlock();
                std::this_thread::sleep_for(std::chrono::microseconds(20));
                lk.lock();
            }
        }
    }
}

void release_server(rc_server* s) {
    // Teardown: failures here have no one left to report to.
    for (Slot& sl : s->slots) {
        if (sl.ev) (void)hipEventDestroy(sl.ev);
        if (sl.d_counters) (void)hipFree(sl.d_counters);
        if (sl.h_reqs) (void)hipHostFree(sl.h_reqs);
        if (sl.h_tiles) (void)hipHostFree(sl.h_tiles);
    }
    for (hipEvent_t e : s->event_pool) (void)hipEventDestroy(e);
    if (s->s_in) (void)hipStreamDestroy(s->s_in);
    if (s->s_comp) (void)hipStreamDestroy(s->s_comp);
    if (s->s_out) (void)hipStreamDestroy(s->s_out);
    if (s->arena_base) (void)hipFree(s->arena_base);
    delete s;
}

}  // namespace

extern "C" {

rc_status rc_server_create(const rc_server_opts* o, rc_server** out) {
    if (!out) return RC_EINVAL;
    *out = nullptr;
    rc_server_opts opts{};
    if (o) opts = *o;
    if (opts.max_jobs < 0 || opts.max_quantum_tiles < 0 || opts.piece_pixels < 0 ||
        opts.reserved != 0)
        return RC_EINVAL;
    if (opts.max_jobs == 0) opts.max_jobs = 64;
    if (opts.max_quantum_tiles == 0) opts.max_quantum_tiles = 4096;
    if (opts.piece_pixels == 0) opts.piece_pixels = (int64_t)16 << 20;
    int dev = 0;
    const DeviceInfo* di = current_device(&dev);
    if (!di) return RC_EHIP;
    rc_server* s = new (std::nothrow) rc_server();
    if (!s) return RC_ENOMEM;
    s->device = dev;
    s->di = di;
    s->lds = std::min(kBatchLds, di->lds);
    s->grid = std::max(1, di->cus) *
              (int)std::max<size_t>(1, std::min<size_t>(kBatchPerCu, di->lds_per_cu / s->lds));
    hipError_t e = hipSuccess;
    auto fail = [&](hipError_t err) {
        release_server(s);
        return err == hipErrorOutOfMemory ? RC_ENOMEM : hip_fail(err);
    };
    if (opts.arena_bytes == 0) {
        size_t fr = 0, tot = 0;
        if ((e = hipMemGetInfo(&fr, &tot)) != hipSuccess) return fail(e);
        opts.arena_bytes = fr / 2;
    }
    s->opts = opts;
    if ((e = hipMalloc(&s->arena_base, opts.arena_bytes)) != hipSuccess) return fail(e);
    s->arena.init(opts.arena_bytes);
    if ((e = hipStreamCreateWithFlags(&s->s_in, hipStreamNonBlocking)) != hipSuccess ||
        (e = hipStreamCreateWithFlags(&s->s_comp, hipStreamNonBlocking)) != hipSuccess ||
        (e = hipStreamCreateWithFlags(&s->s_out, hipStreamNonBlocking)) != hipSuccess)
        return fail(e);
    for (Slot& sl : s->slots) {
        if ((e = hipMalloc(&sl.d_counters, kBatchCounters * sizeof(unsigned int))) != hipSuccess ||
            (e = hipHostMalloc((void**)&sl.h_reqs, sizeof(BatchReq) * opts.max_jobs, 0)) !=
                hipSuccess ||
            (e = hipHostMalloc((void**)&sl.h_tiles, sizeof(BatchTile) * opts.max_quantum_tiles,
                               0)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming)) != hipSuccess ||
            (e = hipMemsetAsync(sl.d_counters, 0, kBatchCounters * sizeof(unsigned int), s->s_comp)) !=
                hipSuccess ||
            (e = hipHostGetDevicePointer((void**)&sl.k_reqs, sl.h_reqs, 0)) != hipSuccess ||
            (e = hipHostGetDevicePointer((void**)&sl.k_tiles, sl.h_tiles, 0)) != hipSuccess)
            return fail(e);
    }
    if ((e = hipStreamSynchronize(s->s_comp)) != hipSuccess) return fail(e);
    if ((e = prepare_batch_kernel(s->lds)) != hipSuccess) return fail(e);
    try {
        s->thread = std::thread(scheduler, s);
    } catch (...) {
        release_server(s);
        return RC_ENOMEM;
    }
    *out = s;
    return RC_OK;
}

rc_status rc_server_submit(rc_server* s, const rc_host_job* j, uint64_t* job_id) {
    if (!s || !j || !job_id) return RC_EINVAL;
    const rc_status st = validate_job(*j);
    if (st != RC_OK) return st;
    auto jp = std::make_shared<Job>();
    jp->host = *j;
    jp->rows = (int64_t)j->bands * j->detectors;
    jp->pixels = jp->rows * j->lines;
    jp->lut_n = jp->rows * j->levels;
    if (jp->pixels > 0) jp->direct_out = mapped_host(j->out, (size_t)jp->pixels * 2);
    size_t a, b, c;
    jp->bytes = job_bytes(*j, jp->direct_out != nullptr, &a, &b, &c);
    jp->submit_s = now_s();
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return RC_ECLOSED;
    if (s->failed) return RC_EHIP;
    if (jp->bytes > s->arena.total()) return RC_ENOMEM;  // can never be admitted
    jp->id = s->next_id++;
    s->jobs[jp->id] = jp;
    s->pending.push_back(jp);
    s->stats.submitted += 1;
    if (jp->direct_out) s->stats.direct_out += 1;
    *job_id = jp->id;
    s->cv_work.notify_one();
    return RC_OK;
}

static void fill_stats(const Job& j, rc_job_stats* st) {
    if (!st) return;
    st->submit_s = j.submit_s;
    st->admit_s = j.admit_s;
    st->start_s = j.start_s;
    st->done_s = j.done_s;
    st->latency_s = j.done_s - j.submit_s;
    st->pixels = j.pixels;
    st->status = j.status;
    st->reserved = 0;
}

rc_status rc_server_wait(rc_server* s, uint64_t job_id, rc_job_stats* st) {
    if (!s) return RC_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->jobs.find(job_id);
    if (it == s->jobs.end()) return RC_EINVAL;
    std::shared_ptr<Job> jp = it->second;
    ++s->waiters;
    s->cv_done.wait(lk, [&] { return jp->done; });
    --s->waiters;
    fill_stats(*jp, st);
    s->jobs.erase(job_id);
    s->cv_done.notify_all();  // rc_server_destroy may be waiting for waiters to leave
    return (rc_status)jp->status;
}

rc_status rc_server_poll(rc_server* s, uint64_t job_id, rc_job_stats* st) {
    if (!s) return RC_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(job_id);
    if (it == s->jobs.end()) return RC_EINVAL;
    std::shared_ptr<Job> jp = it->second;
    if (!jp->done) return RC_EBUSY;
    fill_stats(*jp, st);
    s->jobs.erase(job_id);
    return (rc_status)jp->status;
}

rc_status rc_server_info(rc_server* s, rc_server_stats* st) {
    if (!s || !st) return RC_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    *st = s->stats;
    st->arena_bytes = s->arena.total();
    st->arena_used = s->arena.used();
    st->pending = (int32_t)s->pending.size();
    st->active = (int32_t)s->active.size();
    st->waiters = s->waiters;
    return RC_OK;
}

void rc_server_destroy(rc_server* s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv_work.notify_all();
    }
    if (s->thread.joinable()) s->thread.join();
    (void)hipStreamSynchronize(s->s_in);
    (void)hipStreamSynchronize(s->s_comp);
    (void)hipStreamSynchronize(s->s_out);
    {
        // Every job is finished now (completed or refused): let the threads
        // still inside rc_server_wait return before the server is freed.
        std::unique_lock<std::mutex> lk(s->mu);
        s->cv_done.notify_all();
        s->cv_done.wait(lk, [&] { return s->waiters == 0; });
    }
    release_server(s);
}

void* rc_host_alloc(size_t bytes) {
    void* p = nullptr;
    if (hipHostMalloc(&p, bytes ? bytes : 1, 0) != hipSuccess) return nullptr;
    return p;
}

void rc_host_free(void* p) {
    if (p) (void)hipHostFree(p);
}

}  // extern "C"
