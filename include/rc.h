/*
 * rc.h - radiometric LUT correction on MI355X (gfx950): C ABI of librc.so.
 *
 * The paper (Banerjee & Dave, "GPGPU Based Parallelized Client-Server
 * Framework for Providing High Performance Computation Support", §I) names
 * look-up-table generation and image correction as a typical task that a
 * client submits with its data to a GPU server and gets back. It gives no
 * formula; this library fixes the operation as:
 *
 *   LUT build   lut[b][d][v] = clamp(round_half_away(P_bd(v)), 0, L-1),  v in [0, L)
 *               P_bd(v) = ((a3 v + a2) v + a1) v + a0 in binary64, evaluated in
 *               exactly this order with one rounding per operation (no FMA).
 *               The clamp happens in binary64 before the integer conversion:
 *               NaN, -0, negatives and -Inf give 0; values >= L-1 and +Inf give L-1.
 *   Correction  out[b][n][d] = lut[b][d][min(dn[b][n][d], L-1)]   (a pure gather)
 *
 * Layouts (all dense, row-major, no padding):
 *   coeffs  [bands][detectors][RC_NCOEF] binary64, ascending degree a0..a3;
 *           quadratics pass a3 = 0 (bit-identical to quadratic Horner).
 *   lut     [bands][detectors][levels] uint16.
 *   dn, out [bands][lines][detectors] uint16, band-sequential push-broom
 *           images: one line is one read-out of the detector array.
 *
 * Common rules for every entry point:
 *   - Pointers are device pointers (hipMalloc / torch CUDA tensors) unless a
 *     function says host. The caller owns them. The plain entry points
 *     (rc_lut_build, rc_correct, rc_correct_plan) allocate nothing and never
 *     synchronise, so they can be captured in a hipGraph.
 *   - Arguments are validated on the host before anything is enqueued; on
 *     RC_EINVAL nothing was enqueued. A dimension of 0 is a valid empty call
 *     (RC_OK, nothing enqueued, pointers may then be NULL); negative
 *     dimensions are invalid.
 *   - A failed launch returns RC_EHIP; rc_last_hip_error() gives the
 *     hipError_t (thread-local). Faults inside a kernel surface at the
 *     caller's next synchronisation of `stream`.
 *   - `stream` orders the work; 0 is the null stream.
 *   - Every call is bit-exact against the CPU definition above.
 */
#ifndef RC_H_
#define RC_H_

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RC_OK = 0,
    RC_EINVAL = 1,   /* bad argument; nothing enqueued */
    RC_ENOMEM = 2,   /* an allocation failed or a job can never fit */
    RC_EHIP = 3,     /* a HIP runtime call failed; see rc_last_hip_error() */
    RC_EBUSY = 4,    /* resource temporarily unavailable (retry) */
    RC_ECLOSED = 5   /* the server is shut down */
} rc_status;

#define RC_NCOEF 4
#define RC_LEVELS_MIN 2
#define RC_LEVELS_MAX 65536

/* Human-readable name of a status code (static storage). */
const char* rc_status_str(rc_status s);

/* hipError_t of the last RC_EHIP returned on this thread (0 if none). */
int32_t rc_last_hip_error(void);

/*
 * LUT build (LUT generation, a task named in §I).
 *   coeffs    device, [bands][detectors][4] binary64, 8-byte aligned.
 *   levels    L in [RC_LEVELS_MIN, RC_LEVELS_MAX].
 *   lut       device, [bands][detectors][levels] uint16, 2-byte aligned; written.
 * Errors: RC_EINVAL for NULL pointers with a non-empty size, negative dims,
 * levels out of range, misalignment, byte counts overflowing int64, or lut
 * overlapping coeffs.
 */
rc_status rc_lut_build(const double* coeffs, int32_t bands, int32_t detectors, int32_t levels,
                       uint16_t* lut, hipStream_t stream);

/*
 * Image correction (the task §I pairs with LUT generation) with the library's plan for this
 * shape (a tuned plan from the plan cache if one matches, else the default).
 *   dn        device, [bands][lines][detectors] uint16, 2-byte aligned; read.
 *   lut       device, [bands][detectors][levels] uint16, built by rc_lut_build.
 *   out       device, same shape as dn; written. out == dn (in place) is
 *             allowed; any other overlap of out with dn or lut is RC_EINVAL.
 * Deviation from the two-call outline (dn, lut, lines, detectors, bands, out,
 * stream): `levels` is inserted after `bands` because it is the LUT row pitch.
 */
rc_status rc_correct(const uint16_t* dn, const uint16_t* lut, int64_t lines, int32_t detectors,
                     int32_t bands, int32_t levels, uint16_t* out, hipStream_t stream);

/* ---- execution plans (launch shape of the correction kernel) ---------------------------- */

typedef enum {
    RC_PATH_LDS = 0,    /* strip LUT rows staged in LDS as 16-bit entries, level-major */
    RC_PATH_L2 = 1,     /* gathers from the global LUT, tiles ordered to stay L2-resident */
    RC_PATH_PACKED = 2, /* strip LUT rows staged in LDS as 32-level blocks of a 16-bit base
                           plus 2-bit steps (2.5 bits/entry, exact); a tile whose rows have a
                           step outside 0..3 gathers from the global LUT instead */
    RC_PATH_DENSE = 3   /* strip LUT rows staged in LDS as 64-level blocks of a 16-bit header
                           plus one bit per step (slope s in 0..1: each step s or s + 1),
                           saturated runs extrapolated and clamped back (1.25 bits/entry,
                           exact; levels <= 8192, at most 512 threads); the levels of a block
                           that does not fit this form (decreasing, or steps spread over more
                           than two values, or steps of 3 or more between unsaturated
                           entries) are read from the global LUT instead */
} rc_path;

typedef struct {
    int32_t path;        /* rc_path */
    int32_t strip;       /* W: widest strip, power of two in [1, 1024]; the LDS tile is sized
                            for W detectors */
    int32_t vec;         /* pixels per lane per line: 1, 2, 4 or 8 (8: 16-byte image accesses,
                            needs detectors % 8 == 0 and 16-byte aligned dn and out) */
    int32_t threads;     /* threads that stream the image: 256, 512 or 1024 (RC_PATH_DENSE: 256
                            or 512). When there are no more tiles than CUs, RC_PATH_LDS and
                            RC_PATH_PACKED tiles launch 1024 threads and RC_PATH_DENSE tiles 512;
                            the waves beyond `threads` only help stage the strip */
    int32_t unroll;      /* lines in flight per lane: 4, 8 or 16 */
    int32_t chunk_lines; /* lines per tile, >= 1; with an LDS path and a band whose bytes
                            fit 32-bit offsets, a strip's ceil(lines / chunk_lines) tiles
                            take its passes of lines in turn instead of contiguous ranges */
    int32_t xcd_remap;   /* 1: place neighbouring tiles on the same XCD */
    int32_t nontemporal; /* image cache policy: 0 default, 1 non-temporal loads and stores,
                            2 non-temporal stores, 3 sc0 loads + non-temporal stores,
                            4 sc1 loads + non-temporal stores, 5 sc0 loads */
    int32_t strips;      /* strips per band. 0: ceil(detectors / W) strips of W detectors (the
                            last one narrower). > 0: exactly this many strips of nearly equal
                            width (multiples of vec, each at most W), so that the tile count
                            bands * strips * line chunks can match the device's resident
                            workgroups: every workgroup then streams the same share of the
                            image and stages its LUT strip once */
    int32_t lane_map;    /* 0: W / vec lanes per strip line (a wave covers whole line segments
                            when W / vec divides 64; lanes past a narrower strip idle);
                            1: (strip width) / vec lanes per line, no idle lanes in a wave */
} rc_plan;

/*
 * The plan rc_correct uses for this shape (tuned if the plan cache has one,
 * else the default heuristic). Host only; enqueues nothing.
 * `source` (may be NULL) receives 1 for a tuned plan, 0 for the default.
 */
rc_status rc_plan_for(int64_t lines, int32_t detectors, int32_t bands, int32_t levels,
                      const uint16_t* dn, const uint16_t* out, rc_plan* plan, int32_t* source);

/*
 * rc_correct with an explicit plan. Checks the plan against the shape and the
 * device (LDS size, alignment needed by `vec`): RC_EINVAL if it cannot run.
 * Used by the autotuner and by tests that force a path.
 */
rc_status rc_correct_plan(const uint16_t* dn, const uint16_t* lut, int64_t lines,
                          int32_t detectors, int32_t bands, int32_t levels, uint16_t* out,
                          const rc_plan* plan, hipStream_t stream);

/* ---- streaming ceiling: a plain device copy ------------------------------------------- */

/*
 * Launch shape of rc_stream_copy: workgroup size (256, 512 or 1024), 16-byte
 * loads in flight per lane before the first store (2, 4 or 8), cache policy
 * (0 default, 1 non-temporal loads and stores, 2 non-temporal stores) and
 * resident workgroups per CU (threads * wgs_per_cu <= 2048).
 */
typedef struct {
    int32_t threads;
    int32_t unroll;
    int32_t policy;
    int32_t wgs_per_cu;
} rc_copy_plan;

/*
 * Copies `bytes` bytes from src to dst on the device, with the access width
 * (16 bytes per lane) and cache policies the correction kernels use: the
 * practical ceiling of a stream that reads and writes the same bytes, which
 * is what correcting an image moves apart from its LUT. Not part of the
 * paper's task; the benchmark measures the correction against it.
 *   src, dst  device, 16-byte aligned, not overlapping; caller-owned.
 *   plan      NULL: 256 threads, 4 loads in flight, non-temporal, 8 per CU.
 * Allocates nothing, never synchronises (capturable). RC_EINVAL for NULL or
 * misaligned pointers with bytes > 0, overlap, or a plan outside the ranges
 * above; RC_EHIP if the launch fails. bytes == 0: RC_OK, nothing enqueued.
 */
rc_status rc_stream_copy(const void* src, void* dst, size_t bytes, const rc_copy_plan* plan,
                         hipStream_t stream);

/* ---- correction with a workspace ------------------------------------------------------ */

/*
 * Workspace bytes rc_correct_ws needs for this shape: bands * ceil(levels /
 * 64) * detectors * 10 bytes (rounded up to 256-byte pieces) when 2048 <=
 * levels <= 8192, else 0 (no workspace used). Host only.
 */
size_t rc_correct_ws_bytes(int32_t detectors, int32_t bands, int32_t levels);

/*
 * The correction of rc_correct (same definition, same result bit for bit),
 * for long LUT rows (2048 <= levels <= 8192) in two kernels: the first
 * encodes every 64-level block of every LUT row into the dense form of
 * RC_PATH_DENSE in the workspace (once for the whole LUT, on every CU), the
 * second corrects with tiles that copy their strip's encoded blocks into LDS
 * instead of encoding them (a strip split into line chunks is encoded once,
 * not once per chunk). Other level counts: exactly rc_correct, ws ignored.
 *   ws, ws_bytes  device workspace, 256-byte aligned, ws_bytes >=
 *                 rc_correct_ws_bytes(...); caller-owned, contents
 *                 overwritten, must not overlap dn, out or lut.
 *   plan          NULL: the library's plan; else a RC_PATH_DENSE plan
 *                 (validated as for rc_correct_plan).
 * Allocates nothing, never synchronises (capturable). Two calls that share
 * a workspace must be ordered (one stream): a later call overwrites it.
 * Errors: as rc_correct; RC_EINVAL also for a missing, misaligned, short or
 * overlapping workspace, or a plan that is not RC_PATH_DENSE.
 */
rc_status rc_correct_ws(const uint16_t* dn, const uint16_t* lut, int64_t lines, int32_t detectors,
                        int32_t bands, int32_t levels, uint16_t* out, void* ws, size_t ws_bytes,
                        const rc_plan* plan, hipStream_t stream);

/*
 * LUT generation (§I "LUT generation") that also leaves the LUT's dense
 * encoding in a workspace: the same LUT as rc_lut_build, bit for bit, and
 * the same workspace contents rc_correct_ws writes for that LUT, in one
 * kernel (one wave per LUT row evaluates it, stores it, and encodes its
 * 64-level blocks), so that rc_correct_pre can correct without reading the
 * LUT back. For 2048 <= levels <= 8192 (rc_correct_ws_bytes(...) > 0).
 *   coeffs, lut   as rc_lut_build.
 *   ws, ws_bytes  device workspace, 256-byte aligned, ws_bytes >=
 *                 rc_correct_ws_bytes(detectors, bands, levels); caller-owned,
 *                 contents overwritten, must not overlap coeffs or lut.
 * Allocates nothing, never synchronises (capturable).
 * Errors: as rc_lut_build; RC_EINVAL also for levels outside [2048, 8192]
 * and for a missing, misaligned, short or overlapping workspace.
 */
rc_status rc_lut_build_ws(const double* coeffs, int32_t bands, int32_t detectors, int32_t levels,
                          uint16_t* lut, void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * rc_correct_ws without its encoding pass (§I "Image Correction"): the
 * workspace must already hold the dense encoding of this lut, as
 * rc_lut_build_ws or rc_correct_ws left it (and nothing may have changed the
 * LUT or the workspace since); the result is then rc_correct's, bit for bit.
 * The tiles read the encoded blocks, and the LUT only for levels of blocks
 * the dense form cannot hold. Arguments, plan, ordering and errors as
 * rc_correct_ws; RC_EINVAL also for levels outside [2048, 8192]. A workspace
 * that does not hold the encoding of `lut` gives wrong output, not an error.
 */
rc_status rc_correct_pre(const uint16_t* dn, const uint16_t* lut, int64_t lines, int32_t detectors,
                         int32_t bands, int32_t levels, uint16_t* out, const void* ws,
                         size_t ws_bytes, const rc_plan* plan, hipStream_t stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * correction of rc_correct_ws with the library's own scratch instead of a
 * workspace argument. The scratch is a device array of
 * RC_NOALLOC_SCRATCH_BYTES per GPU, held by the library until the process
 * ends; this call allocates nothing (no hipMalloc, no allocating library
 * routine) and never synchronises. Shapes that rc_correct_ws runs without a
 * workspace run as rc_correct. RC_EINVAL when the shape needs more scratch
 * than RC_NOALLOC_SCRATCH_BYTES (rc_correct_ws_bytes(...) > the maximum),
 * otherwise errors as rc_correct_ws. Every call on one GPU shares its
 * scratch: calls that overlap on one GPU (different streams, or threads
 * without ordering) race and give wrong results; calls ordered on one stream
 * are safe.
 */
#define RC_NOALLOC_SCRATCH_BYTES (32u << 20)
rc_status rc_correct_noalloc(const uint16_t* dn, const uint16_t* lut, int64_t lines,
                             int32_t detectors, int32_t bands, int32_t levels, uint16_t* out,
                             hipStream_t stream);

/* ---- least-squares calibration fit ---------------------------------------------------- */

/*
 * The calibration step upstream of rc_lut_build: case study 2 of the paper
 * (§III.B, least-squares curve fit of any order), applied per band b and
 * detector d to that detector's responses on `points` calibration lines.
 * Fits f(x) = a0 + a1 x + ... + a_m x^m, m = order, to the pairs
 * (x[b][i][d], y[b][i]), i < points, minimising sum_i (y_i - f(x_i))^2 through
 * the normal equations A a = B, A[j][k] = sum_i x_i^(j+k) (A[0][0] = points),
 * B[j] = sum_i x_i^j y_i, solved as a = A^-1 B with A^-1 from Gauss-Jordan
 * elimination with partial pivoting. Binary64, no fused multiply-add, powers
 * by repeated multiplication and sums in point order: every detector's
 * result is a fixed sequence of IEEE operations (bit-identical to a CPU that
 * follows the same steps). The normal equations are ill-conditioned for
 * large x and high orders (cond(A) ~ 1e12 for order 2 over a 10-bit range);
 * the fit is the paper's, not a re-scaled one.
 *
 *   x       device, [bands][points][detectors] binary64 (detector responses)
 *   y       device, [bands][points] binary64 (reference level of each line)
 *   coeffs  device, [bands][detectors][4] binary64, written: a0..a_m, then +0.0
 *           above the order (the layout rc_lut_build reads); all four NaN when
 *           elimination meets no nonzero pivot (e.g. every x_i equal, order >= 1)
 *   order   0..3;  points >= order + 1
 *
 * The caller owns all buffers; nothing is allocated; one kernel is enqueued on
 * `stream`. RC_EINVAL (nothing enqueued) for order outside 0..3, points <
 * order + 1, negative sizes, null or not 8-byte-aligned pointers when there
 * is work, or coeffs overlapping x or y. Zero bands or detectors: RC_OK, no
 * work.
 */
rc_status rc_fit(const double* x, const double* y, int32_t bands, int32_t points,
                 int32_t detectors, int32_t order, double* coeffs, hipStream_t stream);

/* ---- bilinear Bayer demosaicing ------------------------------------------------------- */

/*
 * Case study 1 of the paper (§III.A, bilinear interpolation based
 * demosaicing). raw holds `images` mosaics of height x width 16-bit samples
 * behind an RGGB colour filter (R at even row and even column, B at odd row
 * and odd column, G elsewhere). Each output pixel keeps its own sample for
 * its own colour; each missing colour is the average of that colour's
 * samples among the pixel's 8 direct neighbours, rounded half up in
 * integers: at R and B pixels, G from the 4 cross neighbours and the other
 * of R/B from the 4 diagonal ones; at G pixels, the colour of its row from
 * the 2 horizontal neighbours and the other from the 2 vertical ones. Rows
 * and columns outside the image are mirrored about the edge sample (index -1
 * reads 1, index n reads n - 2), which keeps the colour pattern. Exact
 * integer arithmetic: results are bit-identical to any implementation of this
 * definition.
 *
 *   raw     device, [images][height][width] uint16
 *   rgb     device, [images][3][height][width] uint16, written (R, G, B planes)
 *   height  even, >= 2;  width a multiple of 4, >= 4
 *
 * The caller owns both buffers (8-byte aligned, not overlapping); nothing is
 * allocated; one kernel is enqueued on `stream`. RC_EINVAL (nothing enqueued)
 * for negative sizes, odd height, width not a multiple of 4, null or
 * misaligned pointers when there is work, overlap, or sizes that overflow.
 * Zero images or an empty image: RC_OK, no work.
 */
rc_status rc_demosaic(const uint16_t* raw, int32_t images, int32_t height, int32_t width,
                      uint16_t* rgb, hipStream_t stream);

/* ---- gradient-based Bayer demosaicing ------------------------------------------------- */

/*
 * The gradient interpolation based demosaicing the paper lists beside the
 * bilinear one (§II, §III.A), which it names without giving steps; the method
 * is Hamilton and Adams' adaptive colour plane interpolation (U.S. Patent
 * 5,629,734). Same mosaic, layout and mirrored borders as rc_demosaic (index
 * -1 reads 1, -2 reads 2, n reads n - 2, n + 1 reads n - 3). Integer
 * arithmetic, ">>" an arithmetic shift:
 *
 *   green at an R or B pixel with own sample C, green neighbours Gl Gr Gu Gd
 *   and same-colour samples two away Cl Cr Cu Cd:
 *     lh = 2C - Cl - Cr,  lv = 2C - Cu - Cd
 *     dH = |Gl - Gr| + |lh|,  dV = |Gu - Gd| + |lv|
 *     dH < dV: (2 (Gl + Gr) + lh + 2) >> 2;  dV < dH: (2 (Gu + Gd) + lv + 2) >> 2
 *     equal:   (2 (Gl + Gr + Gu + Gd) + lh + lv + 4) >> 3
 *   with G' that green plane (the sample itself at G pixels):
 *     at a G pixel, the colour of its row from the horizontal pair X1, X2 and
 *     the other colour from the vertical pair: (X1 + X2 + 2 G - G'1 - G'2 + 1) >> 1
 *     at an R (B) pixel, B (R) from the diagonal pair with the smaller
 *     |X1 - X2| + |2 G' - G'1 - G'2|, as (X1 + X2 + 2 G' - G'1 - G'2 + 1) >> 1,
 *     or, when both are equal, (X1 + X2 + X3 + X4 + 4 G' - G'1 - G'2 - G'3 - G'4 + 2) >> 2
 *   every interpolated value clamped to [0, 65535].
 *
 * Results are bit-identical to any implementation of this definition.
 *
 *   raw     device, [images][height][width] uint16
 *   rgb     device, [images][3][height][width] uint16, written (R, G, B planes)
 *   height  even, >= 4;  width a multiple of 4, >= 4
 *
 * The caller owns both buffers (8-byte aligned, not overlapping); nothing is
 * allocated; one kernel is enqueued on `stream`. RC_EINVAL (nothing enqueued)
 * for negative sizes, odd height or height 2, width not a multiple of 4, null
 * or misaligned pointers when there is work, overlap, or sizes that overflow.
 * Zero images or an empty image: RC_OK, no work.
 */
rc_status rc_demosaic_gradient(const uint16_t* raw, int32_t images, int32_t height,
                               int32_t width, uint16_t* rgb, hipStream_t stream);

/* ---- autotuner and plan cache --------------------------------------------------------- */

/*
 * Times candidate plans for this shape on the caller's buffers (dn, lut as
 * for rc_correct; `out` is overwritten, must differ from dn) and records the
 * fastest in the in-memory plan cache under the shape class
 * (arch, CU count, levels, ceil(log2 detectors), ceil(log2 lines), bands,
 * usable vector width). effort 0 = reduced candidate set, 1 = full sweep.
 * `best` / `best_us` (may be NULL) receive the winner and its mean time in us.
 * Shapes whose image (4 B per pixel) and LUT take less than 512 MiB, and so
 * would stay cached across back-to-back calls, are timed one call at a time,
 * each after a 512 MiB scratch write that evicts the caches and a copy of the
 * LUT that brings it back (as a preceding rc_lut_build leaves it); that
 * scratch (512 MiB + the LUT size) is allocated for the duration of the call,
 * and if it cannot be, such shapes are timed back to back like larger ones.
 * Synchronises `stream`; not capturable. Errors: RC_EINVAL, RC_EHIP.
 */
rc_status rc_tune(const uint16_t* dn, const uint16_t* lut, int64_t lines, int32_t detectors,
                  int32_t bands, int32_t levels, uint16_t* out, int32_t effort, rc_plan* best,
                  float* best_us, hipStream_t stream);

/* Persist / reload the plan cache (one JSON object per line). path NULL means
 * $RC_TUNE_CACHE, else tune_cache.json next to librc.so, which is also the
 * file loaded on first use. Return the number of entries, or -1 on I/O error
 * (a failed load leaves the cache empty). Host only. */
int32_t rc_tune_save(const char* path);
int32_t rc_tune_load(const char* path);
/* Empty the in-memory cache (rc_correct then uses default plans). */
void rc_tune_clear(void);
int32_t rc_tune_count(void);

/* ---- batched execution of many uneven requests ----------------------------------------- */

/*
 * One correction job, as a client would submit it to the GPU server of the
 * paper's framework (§II): coefficients in, LUT and corrected image out. All
 * pointers are device pointers with the layouts and rules of rc_lut_build /
 * rc_correct (lut is written by the batch).
 */
typedef struct {
    const double* coeffs;  /* [bands][detectors][4] */
    const uint16_t* dn;    /* [bands][lines][detectors] */
    uint16_t* lut;         /* [bands][detectors][levels], written */
    uint16_t* out;         /* [bands][lines][detectors], written; may equal dn */
    int64_t lines;
    int32_t detectors;
    int32_t bands;
    int32_t levels;
    int32_t reserved;      /* must be 0 */
} rc_request;

typedef struct rc_batch rc_batch;

typedef struct {
    int32_t requests;
    int32_t tiles;        /* correction tiles in the persistent kernel's queue */
    int32_t slots;        /* persistent workgroups */
    int32_t graph;        /* 1 if runs replay a captured hipGraph */
    int64_t pixels;
    int64_t lut_entries;
    int32_t tuned;        /* requests whose tile shape came from a batch entry of the plan
                             cache (rc_batch_tune); the others use the plain path's plan */
    int32_t fused;        /* requests whose LUT is written once and never read back: their
                             tiles evaluate the strip in LDS, or a build kernel writes the
                             LUT and its dense encoding, which the tiles stage */
    int64_t lut_gather_entries; /* LUT entries of the other requests (level counts above
                             8192): written by the build kernel, read back by the gather */
} rc_batch_stats;

#define RC_BATCH_NO_GRAPH 1 /* flag: launch the two kernels directly on every run */

/*
 * Plans a batch of n requests on the current device: validates every request
 * (RC_EINVAL as for the plain calls, and also if a buffer written by a
 * request overlaps any other buffer of any request, except a request's out
 * equal to its own dn), picks each request's tile shape (its batch entry of
 * the plan cache, written by rc_batch_tune; else the plain path's plan for
 * the request fitted to the batch kernel), builds the tile queue (longest
 * tiles first), allocates the batch's small device tables and captures the
 * LUT build kernel plus the persistent correction kernel into a hipGraph.
 * Synchronises; not capturable. The request buffers must stay valid until
 * rc_batch_destroy; their contents may change between runs.
 * flags: 0, or RC_BATCH_NO_GRAPH. This argument is an addition to the
 * interface the batching step was specified with (requests, count, handle):
 * it lets callers that capture their own graphs, or cannot, launch directly.
 * Errors: RC_EINVAL, RC_ENOMEM, RC_EHIP.
 */
rc_status rc_batch_create(const rc_request* reqs, int32_t n, int32_t flags, rc_batch** out);

/*
 * Autotunes the batch kernel's tile shape for the shape classes of `reqs`:
 * requests with pixels are grouped by (levels, ceil(log2 detectors), largest
 * usable vector width); for each class, candidate shapes (LDS mode, strip
 * width, pixels per lane) run the class's requests as one batch, launched
 * directly on `stream` (one warm-up run, then 3 timed with HIP events). The
 * shape rc_batch_create would take without an entry runs first and is kept
 * unless a candidate is at least 2 % faster; the result goes into the plan
 * cache as that class's batch entry (rc_tune_save persists it). effort 0
 * tries the two widest strips and two
 * vector widths per LDS mode; effort 1 one more of each. The runs write the
 * requests' lut and out exactly as rc_batch_run would. Validates as
 * rc_batch_create; synchronises; allocates (each candidate's tables).
 * *classes (if not NULL) = classes tuned.
 * Errors: RC_EINVAL, RC_ENOMEM, RC_EHIP.
 */
rc_status rc_batch_tune(const rc_request* reqs, int32_t n, int32_t effort, int32_t* classes,
                        hipStream_t stream);

/* Enqueues one run of the whole batch (LUT build, then correction) on
 * `stream`; no synchronisation, no allocation. Runs on one batch must not
 * overlap in time (they share the tile counters): order them on one stream.
 * RC_EINVAL if the current device is not the batch's. */
rc_status rc_batch_run(rc_batch* b, hipStream_t stream);

rc_status rc_batch_info(const rc_batch* b, rc_batch_stats* stats);

/* Frees the batch (its runs must have completed). NULL is ignored. */
void rc_batch_destroy(rc_batch* b);

/* ---- serving: continuous batching of jobs from host memory ----------------------------- */

/*
 * The paper's framework (§II) lets clients submit a processing task with its
 * data to a remote GPU server and receive the results. An rc_server is that
 * server's GPU side, in-process: jobs arrive at any time with host buffers;
 * a scheduler thread admits each job when its device bytes fit the server's
 * arena and a job slot is free (first come, first served), copies it in
 * piece by piece on a host-to-device stream, runs the tiles of every piece
 * that has arrived, from all admitted jobs together, as quanta of one
 * persistent kernel (continuous batching), and copies each finished piece
 * back on a device-to-host stream. Results are bit-identical to rc_lut_build
 * + rc_correct on the same job.
 */
typedef struct rc_server rc_server;

typedef struct {
    uint64_t arena_bytes;      /* device memory for admitted jobs; 0 = half the free memory */
    int32_t max_jobs;          /* jobs admitted at once; 0 = 64 */
    int32_t max_quantum_tiles; /* tiles per persistent launch; 0 = 4096 */
    int64_t piece_pixels;      /* pixels per copy piece; 0 = 16 Mi */
    int32_t flags;             /* must be 0 */
    int32_t reserved;          /* must be 0 */
} rc_server_opts;

/*
 * A job in host memory. Layouts as for rc_lut_build / rc_correct. Use pinned
 * memory (rc_host_alloc) for full-speed, asynchronous copies; pageable
 * buffers work but make the scheduler wait on each copy. When `out` is one
 * pinned allocation the device can address, the kernel writes the corrected
 * image into it directly (no device copy of the output, no copy back). The
 * caller owns the buffers and must keep them valid, and not modify dn/coeffs
 * or read out, until rc_server_wait or rc_server_poll reports the job
 * finished, with any status: a job failed with RC_EHIP is reported only
 * after the server's streams have drained, so nothing touches its buffers
 * afterwards.
 */
typedef struct {
    const double* coeffs;  /* host, [bands][detectors][4] */
    const uint16_t* dn;    /* host, [bands][lines][detectors] */
    uint16_t* out;         /* host, [bands][lines][detectors], written */
    uint16_t* lut;         /* host, [bands][detectors][levels], written; NULL: not returned */
    int64_t lines;
    int32_t detectors;
    int32_t bands;
    int32_t levels;
    int32_t reserved;      /* must be 0 */
} rc_host_job;

typedef struct {
    double submit_s;   /* host steady-clock seconds: rc_server_submit */
    double admit_s;    /* admitted (device memory reserved, copies in enqueued) */
    double start_s;    /* first tile issued to the GPU */
    double done_s;     /* scheduler saw the last copy back complete */
    double latency_s;  /* done_s - submit_s */
    int64_t pixels;
    int32_t status;    /* rc_status of the job */
    int32_t reserved;
} rc_job_stats;

typedef struct {
    uint64_t submitted, completed;
    uint64_t quanta, tiles;    /* persistent launches and tiles issued */
    uint64_t pixels;           /* pixels of completed jobs */
    uint64_t arena_bytes, arena_used;
    int32_t pending, active;   /* jobs waiting for admission / admitted */
    int32_t waiters;           /* threads blocked in rc_server_wait */
    int32_t direct_out;        /* submitted jobs whose output the kernel writes to host memory */
} rc_server_stats;

/* Creates a server on the current device (arena, streams, scheduler thread).
 * o may be NULL for defaults. Errors: RC_EINVAL, RC_ENOMEM, RC_EHIP. */
rc_status rc_server_create(const rc_server_opts* o, rc_server** out);

/* Queues a job; returns at once with its id. RC_EINVAL for bad jobs,
 * RC_ENOMEM if the job can never fit the arena, RC_ECLOSED after
 * rc_server_destroy began, RC_EHIP if the server failed. */
rc_status rc_server_submit(rc_server* s, const rc_host_job* j, uint64_t* job_id);

/* Blocks until the job finished; returns its status (RC_OK, RC_ECLOSED if the
 * server shut down before admitting it, RC_EHIP on a device error) and fills
 * st (may be NULL). A job id can be waited for (or polled to completion) once. */
rc_status rc_server_wait(rc_server* s, uint64_t job_id, rc_job_stats* st);

/* Non-blocking: RC_EBUSY while the job runs, else as rc_server_wait. */
rc_status rc_server_poll(rc_server* s, uint64_t job_id, rc_job_stats* st);

rc_status rc_server_info(rc_server* s, rc_server_stats* st);

/* Stops admitting, lets admitted jobs finish, completes never-admitted jobs
 * with RC_ECLOSED, then frees everything. Must not race with other calls on s
 * except waiters of its jobs. NULL is ignored. */
void rc_server_destroy(rc_server* s);

/* Pinned host memory for job buffers (hipHostMalloc); NULL on failure. */
void* rc_host_alloc(size_t bytes);
void rc_host_free(void* p);

/* ---- wire front end: the paper's client-server protocol --------------------------------- */

/*
 * The TCP front end of the paper's client-server framework (§II, Fig. 3):
 * a client sends a 260-byte header, then the input data; the server runs the
 * task on the GPU and answers with a header of the same layout followed by
 * the result. Header fields (byte offsets; text fields NUL-padded):
 *
 *   [0, 29)    task flag: "LUT_CORRECTION", "BILINEAR_DEMOSAIC", "GRADIENT_DEMOSAIC",
 *              "LSQ_FIT", "GPU_INFO"
 *   [29]       '+' when data follows the header, '\0' when none does
 *   [30, 230)  comma-separated parameters, key=value
 *   [230, 260) output file name (the client's; echoed back, never opened here)
 *   [260, ...) data, little-endian, laid out as for the C calls:
 *     LUT_CORRECTION     bands=B,lines=N,detectors=D,levels=L[,lut=1]
 *                        in:  coeffs f64 [B][D][4], then dn u16 [B][N][D]
 *                        out: corrected u16 [B][N][D] (then the LUT u16 [B][D][L] if lut=1)
 *     BILINEAR_DEMOSAIC  images=I,height=H,width=W
 *                        in:  raw u16 [I][H][W];  out: rgb u16 [I][3][H][W]
 *     GRADIENT_DEMOSAIC  as BILINEAR_DEMOSAIC (rc_demosaic_gradient; height >= 4)
 *     LSQ_FIT            bands=B,points=n,detectors=D,order=m
 *                        in:  x f64 [B][n][D], then y f64 [B][n];  out: coeffs f64 [B][D][4]
 *     GPU_INFO           no parameters, no data;  out: an XML listing of the device
 * The answer's parameter field reads "status=<rc_status name>,bytes=<result bytes>".
 * Correction jobs of all connections go through one rc_server (continuous
 * batching); the other tasks run on a stream of the connection.
 */
#define RC_WIRE_HEADER_BYTES 260

typedef enum {
    RC_TASK_LUT_CORRECTION = 1,
    RC_TASK_BILINEAR_DEMOSAIC = 2,
    RC_TASK_LSQ_FIT = 3,
    RC_TASK_GPU_INFO = 4,
    RC_TASK_GRADIENT_DEMOSAIC = 5
} rc_task;

typedef struct {
    int32_t task;          /* rc_task */
    int32_t has_data;      /* the '+' flag */
    char task_flag[30];    /* NUL-terminated copies of the text fields */
    char params[201];
    char out_name[31];
    int64_t bands, lines, detectors, levels, points, order, images, height, width;
    int32_t want_lut;
    int32_t reserved;
    uint64_t data_bytes;   /* input bytes that follow the header */
    uint64_t result_bytes; /* bytes of the answer's data */
} rc_wire_request;

/* Parses and validates one request header (host only, no GPU). RC_EINVAL for
 * an unknown task, a missing or malformed parameter, sizes out of range or
 * overflowing, or a '+' flag that does not match the task. */
rc_status rc_wire_parse(const uint8_t* header, rc_wire_request* req);

typedef struct rc_wire rc_wire;

typedef struct {
    int32_t port;            /* TCP port; 0 picks a free one (see rc_wire_port) */
    int32_t any_address;     /* 0: listen on 127.0.0.1 only; 1: on every interface */
    uint64_t max_data_bytes; /* largest accepted request data, and largest result; 0 = 8 GiB */
    uint64_t arena_bytes;    /* device arena of the internal rc_server; 0 = its default */
} rc_wire_opts;

/* Starts listening on the current device (one accept thread, one thread per
 * connection; a connection may send several requests in turn). o may be NULL
 * for defaults. Errors: RC_EINVAL, RC_ENOMEM, RC_EHIP (device), RC_EBUSY
 * (the port cannot be bound). */
rc_status rc_wire_start(const rc_wire_opts* o, rc_wire** out);

/* The port the server listens on (useful with port 0). */
int32_t rc_wire_port(const rc_wire* w);

/* Stops accepting, closes every connection after its current request, joins
 * all threads and frees the server. NULL is ignored. */
void rc_wire_stop(rc_wire* w);

#ifdef __cplusplus
}
#endif

#endif /* RC_H_ */
