/*
 * ff.h -- C ABI of the MI355X (gfx950) Flow Fields dense correspondence search.
 *
 * The search is the matching stage of FlowFields++ (Sec. 3.1 "Matches"):
 * feature descriptors, initial matches at the lowest pyramid resolution,
 * propagation into all four directions with random search at every scale
 * of a coarse-to-fine pyramid, and the forward-backward consistency check
 * with threshold epsilon (Sec. 3.1; Table 3).  Every output is integer and
 * exactly defined:
 *   - luma Y = (77 R + 150 G + 29 B + 128) >> 8 (C = 3) or the input (C = 1);
 *   - pyramid: 2x2 box mean rounded half up, floor dimensions;
 *   - descriptors: the 16 lowest-sequency 2-D Walsh-Hadamard coefficients of
 *     the 8x8 patch (offsets -3..+4, replicated border), floor(c / 64), DC
 *     shifted by -128, as int8;
 *   - cost: SAD of two descriptors, or (FF_COST_CENSUS) the Hamming distance
 *     of two 7x7 Census strings of the luma -- bit k for the k-th of the 48
 *     neighbours in row-major order, set when the neighbour is strictly
 *     darker than the centre, border replicated; INT32_MAX when the target
 *     leaves image B;
 *   - seeds: exact nearest neighbour (squared L2, lowest linear index on
 *     ties) of every stride-grid pixel at the coarsest level among all pixels;
 *   - per level: init (seed of the pixel's stride cell, or twice the parent
 *     flow), then `iters` times: LR, RL sweeps, random search 0, TB sweep,
 *     random search 1, BT sweep, random search 2;
 *   - random search: radii R, R>>1, ..., 1 around the pre-pass flow, offsets
 *     from Philox4x32-10 at counter (y*W+x, level, iter<<2|pass, j>>1) and
 *     key (seed low, seed high), accepted on a strictly lower cost;
 *   - mask(p) = 1 iff both matches are valid and |F(p) + B(p + F(p))|^2 <= eps^2;
 *     with FF_SECOND_CHECK also against B2, the inverse field of the same
 *     search keyed by seed2, the error then being the larger of the two;
 *   - optionally (FF_SPARSIFY, Sec. 3.1 with s from Table 3): in every 3x3
 *     block from the origin (partial at the borders) holding at least s
 *     consistent matches, only the match with the lowest consistency error
 *     |F(p) + B(p + F(p))|^2 is kept (the lowest y*W + x among equals).
 *
 * Memory: every pointer in ff_pair is DEVICE memory owned by the caller.
 * The handle owns its workspaces (pyramids, descriptors, search state, seed
 * tables), allocated on first use for a shape/batch and reused after.
 * Calls are stream-ordered: they validate synchronously, enqueue the work on
 * `stream` (a hipStream_t, or NULL for the null stream) and return; outputs
 * are valid once the stream reaches that point.  Calls on one handle share
 * its workspace, so a call on a different stream than the handle's previous
 * call first makes its stream wait for that call's work (an event): calls
 * on one handle never overlap on the device, whatever their streams.  A
 * handle must not be used from two threads at once.  Errors of
 * already-enqueued work surface as FF_ERR_HIP on a later call.
 *
 * Budget: params.hbm_budget caps the device memory a handle holds -- its
 * own workspace (ff_match_pair / ff_match_batch) and its serving lanes
 * together.
 */
#ifndef FF_H
#define FF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ff_ctx* ff_handle;

typedef enum {
    FF_OK = 0,
    FF_ERR_INVALID = 1,      /* bad argument: NULL pointer, size, parameter  */
    FF_ERR_OOM = 2,          /* device allocation failed                    */
    FF_ERR_BUDGET = 3,       /* workspace would exceed params.hbm_budget     */
    FF_ERR_HIP = 4,          /* a HIP runtime call failed (see ff_last_error) */
    FF_ERR_UNSUPPORTED = 5,  /* device is not gfx950                         */
    FF_ERR_BUSY = 6          /* serving queue full                           */
} ff_status;

/* flags */
#define FF_SPARSIFY 1u      /* compute sparse_fwd / sparse_bwd (3x3-block selection) */
#define FF_COST_CENSUS 2u   /* matching cost = Hamming distance of 7x7 Census strings
                               (Sec. 3.1) instead of descriptor SAD; seeds still
                               match descriptors; staged schedules (mode 1)
                               unsupported                                         */
#define FF_SECOND_CHECK 4u  /* two consistency checks (Sec. 3.1): the search runs a
                               second time keyed by seed2, and a match must also be
                               consistent with that search's inverse field        */
#define FF_SECOND_PARAMS 16u /* with FF_SECOND_CHECK: the second search also runs
                               with its own matching parameters (Sec. 3.1: the
                               inverse fields of the two checks come from
                               searches with different parameters) -- iters2
                               iterations per level and random-search radius
                               rs_radius2 -- instead of the first search's   */
#define FF_SUBPIXEL 8u      /* sub-pixel refinement (Sec. 3.1): after the integer
                               search, sub_iters more iterations at level 0 on flows
                               in quarter pixels, the cost of a quarter-pixel target
                               taken on B's descriptors interpolated bilinearly
                               (integer weights (4-ax)(4-ay), ax(4-ay), (4-ax)ay,
                               ax ay over the biased bytes, (sum + 8) >> 4); flow
                               outputs then in quarter pixels, fberr in 1/16 px^2,
                               the consistency target rounded half up to whole
                               pixels; descriptor cost only; W, H <= 2048; the
                               refinement runs a fixed schedule ((1, 8, 0) rows,
                               (1, 4, 0) columns) whatever the tuning            */

/* Search parameters (Sec. 3.1; Table 3 gives epsilon = 1 and s = 7 for
 * KITTI, epsilon = 7 and s = 4 for MPI Sintel). */
typedef struct {
    int32_t  levels;        /* pyramid levels L, 1..8 (3 or 4 in the workloads)  */
    int32_t  seed_stride;   /* seed grid step at the coarsest level, 1..64 (3)   */
    int32_t  iters;         /* iterations per level, 0..64 (2)                   */
    int32_t  rs_radius;     /* random-search radius R, 0..1024 (16)              */
    int32_t  fb_eps;        /* consistency threshold in px, 0..1024 (1)          */
    uint64_t seed;          /* random-search key                                 */
    uint64_t hbm_budget;    /* cap on workspace bytes; 0 = no cap                */
    uint32_t flags;         /* FF_SPARSIFY | FF_COST_CENSUS | FF_SECOND_CHECK |
                               FF_SECOND_PARAMS | FF_SUBPIXEL, or 0            */
    int32_t  sparse_min;    /* s: matches a 3x3 block needs to keep one, 1..9
                               (7); read only with FF_SPARSIFY                 */
    uint64_t seed2;         /* random-search key of the second search; read
                               only with FF_SECOND_CHECK                       */
    int32_t  sub_iters;     /* FF_SUBPIXEL: refinement iterations, 1..16 (1)    */
    int32_t  sub_radius;    /* FF_SUBPIXEL: random-search radius in quarter
                               pixels, 0..64 (2: trials at 1/2 and 1/4 px)     */
    int32_t  iters2;        /* FF_SECOND_PARAMS: the second search's iterations
                               per level, 0..64                               */
    int32_t  rs_radius2;    /* FF_SECOND_PARAMS: its random-search radius,
                               0..1024                                         */
} ff_params;

/* One image pair and its outputs.  Both frames are [H][W][C] uint8,
 * row pitch W*C bytes, C in {1, 3}; 1 <= W, H <= 8192 and
 * min(W, H) >> (levels-1) >= 1.
 * flow_*: [H][W][2] int16 (dx, dy); cost_*: [H][W] int32 (INT32_MAX =
 * no valid match); mask_*: [H][W] uint8 (1 = consistent).  flow_fwd and
 * mask_fwd are required; every other output may be NULL.
 * fberr_*: [H][W] int32 consistency error |F(p) + B(p + F(p))|^2, INT32_MAX
 * where either match is invalid (mask = fberr <= eps^2); written when not
 * NULL.  sparse_*: [H][W] uint8, 1 = match kept by the 3x3-block
 * sparsification; sparse_fwd is required with FF_SPARSIFY, and both must be
 * NULL without it.  flow, cost and fberr buffers must be 4-byte aligned.  */
typedef struct {
    const uint8_t* img1;
    const uint8_t* img2;
    int32_t width, height, channels;
    int16_t* flow_fwd;
    int32_t* cost_fwd;
    uint8_t* mask_fwd;
    int16_t* flow_bwd;
    int32_t* cost_bwd;
    uint8_t* mask_bwd;
    int32_t* fberr_fwd;
    uint8_t* sparse_fwd;
    int32_t* fberr_bwd;
    uint8_t* sparse_bwd;
} ff_pair;

/* Create a handle on HIP device `device` (must be gfx950) for the search
 * parameters of Sec. 3.1 (pyramid depth, seed grid, iterations, random-search
 * radius, consistency threshold epsilon and sparsification minimum s of
 * Table 3).  Copies *params; allocates no device workspace yet (the first
 * call sizes it).  FF_ERR_INVALID for a NULL argument, a device index out of
 * range, a parameter outside the ranges above, an unknown flag, or
 * FF_SUBPIXEL together with FF_COST_CENSUS; FF_ERR_UNSUPPORTED on another
 * architecture; FF_ERR_HIP when the runtime fails.  *out is NULL on error;
 * on success the caller owns the handle until ff_destroy. */
ff_status ff_create(const ff_params* params, int device, ff_handle* out);

/* Match one pair on `stream`: the matching of Sec. 3.1 from the two frames
 * to the outputs of ff_pair -- luma, pyramid, descriptors, exact initial
 * matches at the coarsest level, per level the initialisation and `iters`
 * rounds of propagation in four directions with random search, optionally
 * the quarter-pixel refinement, then the forward-backward consistency check
 * (threshold epsilon, Table 3), optionally the second check and the 3x3
 * sparsification.  All pointers of *pair are caller-owned device memory
 * that must stay valid until the stream has passed the call.
 * FF_ERR_INVALID for a NULL or malformed pair (see ff_pair), FF_ERR_BUDGET
 * when the workspace would exceed the budget, FF_ERR_OOM when the device
 * allocation fails, FF_ERR_HIP when the runtime fails; nothing is enqueued
 * then.  The handle's workspace grows to the largest call and is kept. */
ff_status ff_match_pair(ff_handle h, const ff_pair* pair, void* stream);

/* Match n independent pairs, of any sizes, in one grouped pass (the search
 * of Sec. 3.1 on every pair): every stage runs once over all pairs.
 * Outputs are bit-identical to n calls of ff_match_pair.  1 <= n <= 32767;
 * errors as ff_match_pair (the first invalid pair rejects the batch and
 * nothing is enqueued). */
ff_status ff_match_batch(ff_handle h, const ff_pair* pairs, int32_t n, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * search and bit-identical outputs as ff_match_pair, with the pair's whole
 * workspace in a fixed scratch array of 128 MiB per device inside the
 * library (reserved when the library's code is loaded on a device; a
 * 1242 x 375 pair with every flag needs about 92 MB).  It calls no
 * hipMalloc, hipFree or pinned-memory allocation, captures no graph and
 * records no tracing events.  Calls on one device share the array, which
 * keeps the last call's contents (every buffer is written before it is
 * read); they are ordered through an event, so calls on different streams,
 * handles or host threads of one process run one after the other on the
 * device rather than racing.  FF_ERR_BUDGET when the pair needs more than
 * the array holds (ff_workspace_bytes of the pair + 1 KiB of table); other
 * errors as ff_match_pair. */
ff_status ff_match_pair_noalloc(ff_handle h, const ff_pair* pair, void* stream);

/* Synchronise the handle's device and free everything it owns (workspace,
 * serving lanes, graphs, events).  NULL is ignored.  Not part of the method:
 * resource management. */
void ff_destroy(ff_handle h);

/* Message of the last non-OK status on this handle (static string when h is
 * NULL).  Valid until the next call on the handle.  Not part of the method. */
const char* ff_last_error(ff_handle h);

/* Bytes of device workspace a batch of these pairs needs (no allocation):
 * the pyramids, descriptor planes, search state and seed tables of Sec. 3.1
 * for every pair; only width, height and channels of each pair are read.
 * 0 for a NULL handle or pairs, or n < 1. */
uint64_t ff_workspace_bytes(ff_handle h, const ff_pair* pairs, int32_t n);

/* ---- serving: continuous batching --------------------------------------
 * Deployment of the search of Sec. 3.1 as a request loop; the arithmetic of
 * every pair is that of ff_match_pair.
 * The handle keeps `lanes` concurrent cohorts, each on its own HIP stream
 * with its own preallocated workspace of `lane_bytes` bytes (lanes x
 * lane_bytes, plus the handle's own workspace, must fit params.hbm_budget
 * when a budget is set: ff_serve_config releases the handle's own workspace
 * when both do not fit, and a later ff_match_* regrows it within what the
 * lanes leave, or fails with FF_ERR_BUDGET).  ff_submit
 * queues one pair (FIFO) and returns at once; whenever a lane is idle, the
 * queued pairs at the head that fit its workspace start as one grouped
 * batch on that lane, overlapping with the cohorts running on the others.
 * A pair's outputs are bit-identical to ff_match_pair on the same inputs,
 * whatever cohort it ran in.  The inputs are read after the work the caller
 * enqueued on `stream` before the submit; the caller keeps every buffer of
 * the pair alive until ff_poll has returned its tag, after which the
 * outputs are complete.  ff_match_pair / ff_match_batch on the same handle
 * use a separate workspace.
 *
 * ff_serve_config: (re)configure, 1 <= lanes <= 16, lane_bytes >= 1 MiB;
 *   FF_ERR_BUSY while requests are queued or running.  Without it the first ff_submit configures 4 lanes of
 *   hbm_budget / 4 bytes (4 GiB each when no budget is set).
 * ff_submit: FF_OK once the pair is queued; FF_ERR_BUDGET when the pair
 *   alone exceeds lane_bytes, FF_ERR_INVALID for a bad pair (not queued).
 * ff_poll: non-blocking; writes up to `max` finished tags (completion
 *   order), returns how many, or -1 on error (ff_last_error names it).
 *   A cohort that cannot start (an allocation or launch failure on its
 *   lane) goes back to the head of the queue unchanged, so no submitted
 *   pair is lost: every ff_poll tries again, returning -1 while it fails.
 * ff_serve_inflight: queued + running pairs, or -1.                        */
ff_status ff_serve_config(ff_handle h, int32_t lanes, uint64_t lane_bytes);
ff_status ff_submit(ff_handle h, const ff_pair* pair, uint64_t tag, void* stream);
int32_t   ff_poll(ff_handle h, uint64_t* tags_done, int32_t max);
int32_t   ff_serve_inflight(ff_handle h);

/* ---- schedule autotuning -----------------------------------------------
 * Scheduling of the propagation and random search of Sec. 3.1 only.
 * The row and column phases run one wave per image line and solve each
 * sweep on windows of `chunks` x 64 pixels; blocks hold `lines` waves; the
 * mode says how the waves of a block move: 0, each at its own pace; 2, their
 * windows in lockstep (adjacent lines then share the cache lines of B's
 * neighbourhood); 1, in lockstep and reading random-search trials from an
 * LDS copy of the windows' target neighbourhood.  All three are scheduling
 * choices only: the sweep's result does not depend on the window, and
 * lockstep and staging change when and where a descriptor is read, not
 * which one -- no choice changes any output.  Supported triples: mode 0
 * with chunks in {1,2,4,8} and lines in {2,4,8}; mode 2 with chunks in
 * {1,2} and lines in {2,4,8}; mode 1 with (chunks, lines) in {(1,4), (1,8),
 * (1,16), (2,8)} and the descriptor cost.  ff_autotune runs this batch once
 * per supported triple (twice, the second timed with events) and keeps, per
 * phase and level, the fastest; it synchronises the stream.  ff_tune_get
 * writes 6 * levels int32 (cfg[(phase * levels + level) * 3 + {0: chunks,
 * 1: lines, 2: mode}], phase 0 = row, 1 = column) and returns that count,
 * or -1 if max is too small; ff_tune_set installs such a vector
 * (FF_ERR_INVALID for an unsupported triple).  The default is (1, 4, 0) for
 * the row phase and (1, 8, 0) for the column phase at every level.        */
ff_status ff_autotune(ff_handle h, const ff_pair* pairs, int32_t n, void* stream);
int32_t   ff_tune_get(ff_handle h, int32_t* cfg, int32_t max);
ff_status ff_tune_set(ff_handle h, const int32_t* cfg, int32_t n);

/* ---- per-kernel timing (tracing) ------------------------------------------
 * When enabled, every launch the handle enqueues is bracketed by a pair of
 * HIP events on the launch stream.  ff_profile_read synchronises those
 * events, writes one entry per kernel (launch count and summed device time
 * between its events) into out[0..max), returns the number of entries, and
 * clears the record.  Names: gray, down2, desc, seed_records, seed_nn, init,
 * row_phase, col_phase, transpose, fb, sparse, census, save_state,
 * to_quarter, sub_row_phase, sub_col_phase, seed_resolve.  Returns -1 on
 * error.                                                                    */
typedef struct {
    char    name[32];
    int32_t launches;
    double  total_ms;
} ff_profile_entry;

ff_status ff_profile_enable(ff_handle h, int32_t on);
int32_t   ff_profile_read(ff_handle h, ff_profile_entry* out, int32_t max);

/* ---- intermediates, for parity tests against an independent CPU model ----
 * Each stage names a step of Sec. 3.1 in the order the search takes them. */
typedef enum {
    FF_STAGE_GRAY = 0,      /* image `image` level-0 luma: [H][W] uint8               */
    FF_STAGE_PYRAMID = 1,   /* image `image` level `level`: [H_l][W_l] uint8          */
    FF_STAGE_DESC = 2,      /* image `image` level `level`: [H_l][W_l][16] int8       */
    FF_STAGE_SEEDS = 3,     /* direction `dir`: seed-grid NN index, [nsy][nsx] int32  */
    FF_STAGE_STATE = 4,     /* direction `dir`, level, iter, step: [H_l][W_l] of
                               {int16 dx, int16 dy, int32 cost}; step 0 = after init
                               (iter ignored), 1 LR, 2 RL, 3 RS0, 4 TB, 5 RS1, 6 BT,
                               7 RS2; with FF_SUBPIXEL, level = levels names the
                               refinement (step 0 = flows in quarter pixels)        */
    FF_STAGE_CENSUS = 5     /* image `image` level `level`: [H_l][W_l] uint64 Census
                               strings (handles created with FF_COST_CENSUS)         */
} ff_stage_kind;

typedef struct {
    int32_t kind;           /* ff_stage_kind                     */
    int32_t image;          /* 0 = img1, 1 = img2 (GRAY/PYRAMID/DESC/CENSUS) */
    int32_t dir;            /* 0 = forward, 1 = backward (SEEDS/STATE) */
    int32_t level;
    int32_t iter;
    int32_t step;
} ff_stage;

/* Run the search of one pair up to the named point and copy that
 * intermediate into `dst` (device memory of the size stated above). */
ff_status ff_debug_stage(ff_handle h, const ff_pair* pair, const ff_stage* which,
                         void* dst, void* stream);

/* Allocation fault injection, for tests of the error paths (not part of the
 * method): from now on the first `after` device or pinned allocations the
 * handle makes (its workspace, pair table, staging buffers and serving
 * lanes) succeed and every later one fails as the device being out of
 * memory; after < 0 switches it off.  A call that meets such a failure
 * returns FF_ERR_OOM and leaves the handle usable; what the handle did
 * allocate before the failure stays owned by it (reused by later calls,
 * freed by ff_destroy), so nothing leaks.  The environment variable FF_FAULT_ALLOC_AFTER=n sets
 * the same from ff_create on (which then returns FF_ERR_OOM when its own
 * staging allocation fails).  FF_ERR_INVALID for a NULL handle. */
ff_status ff_debug_fault_alloc(ff_handle h, int64_t after);

#ifdef __cplusplus
}
#endif
#endif /* FF_H */
