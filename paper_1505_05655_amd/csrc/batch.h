// Descriptors and launchers of the persistent tile kernel shared by the batch
// and serving runtimes (internal to librc).
#pragma once

#include <hip/hip_runtime_api.h>
#include <stddef.h>
#include <stdint.h>

#include "rc.h"

namespace rc {

constexpr int kBatchThreads = 1024;
constexpr int kBatchUnroll = 4;
constexpr size_t kBatchLds = 80 * 1024;
// Resident workgroups per CU the batch launch aims for (2048 threads per CU).
constexpr int kBatchPerCu = 2048 / kBatchThreads;
// Tile queues of the persistent kernel: one per XCD (workgroups are dispatched
// to the XCDs round-robin, so workgroup i starts on queue i % kBatchQueues).
constexpr int kBatchQueues = 8;
// Device counters of one launch: a head per queue, then the number of
// workgroups that have finished.
constexpr int kBatchCounters = kBatchQueues + 1;

// Per-request descriptor, resident in device memory.
struct BatchReq {
    const double* coeffs;
    const uint16_t* dn;
    uint16_t* lut;
    uint16_t* out;
    int64_t lines;
    int32_t detectors;
    int32_t bands;
    int32_t levels;
    int32_t log_strip;
    int32_t vec;
    int32_t mode;     // kRaw / kGlobal / kPacked / kDense
    int32_t lut_vec;  // LUT rows allow 16-byte loads/stores
    int32_t fused;    // tiles build their LUT strip in LDS (kRaw / kPacked)
    int32_t pad;
    // kDense: the request's dense workspace, [bands][blocks][detectors]
    // planes and headers, written by k_batch_encode before the tiles run.
    uint64_t* planes;
    int16_t* heads;
};

struct BatchTile {
    int32_t req;
    int32_t band;
    int32_t d0;
    int32_t pad;
    int64_t n0;
    int64_t n1;
};

// Queue q holds tiles [bound[q], bound[q + 1]); bound is non-decreasing from
// 0 to the tile count. A single queue is bound = {0, n, n, ..., n}.
struct BatchQueues {
    int32_t bound[kBatchQueues + 1];
};

// Persistent correction kernel: each of the `grid` workgroups pops tiles
// from its own queue, then from the others until every queue is empty.
// `counters` holds kBatchCounters zeros before the first launch; the kernel
// rearms them itself.
hipError_t launch_batch_apply(const BatchReq* reqs, const BatchTile* tiles,
                              const BatchQueues& queues, unsigned int* counters, int grid,
                              size_t lds, hipStream_t stream);

// Queues holding tiles [0, n) in one queue.
BatchQueues single_queue(int32_t n);

// Sets the persistent kernel's dynamic LDS limit on the current device.
hipError_t prepare_batch_kernel(size_t lds);

// Fills q's strip shape and mode from a plain-path plan, fitted to the
// persistent kernel's workgroup size and LDS budget. Dense plans keep the
// dense mode only if allow_dense (the caller then provides the request's
// dense workspace and runs k_batch_encode first); otherwise they become
// packed.
void fit_request_plan(const rc_plan& plan, int levels, size_t lds_cap, bool allow_dense,
                      BatchReq* q);

}  // namespace rc
