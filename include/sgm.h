/*
 * sgm.h - C ABI of an MI355X (gfx950) implementation of the Semi-Global
 * Matching disparity pipeline of Hernandez-Juarez et al., "Embedded
 * real-time stereo estimation via Semi-Global Matching on the GPU"
 * (arXiv 1610.04121).
 *
 * Pipeline (Sec. 2): census-transform features of both images (Sec. 3.1,
 * Eq. 1), Hamming matching cost (Eq. 2), cost aggregation along 2, 4 or 8
 * path directions with the recurrence of Eq. 3, summation over directions and
 * winner-take-all (Eq. 4), a 3x3 median (Sec. 2, stage 4) and, optionally, a
 * left-right consistency check (named as a post-filter in Sec. 5).
 *
 * Conventions shared by every call:
 *  - Image and disparity pointers are DEVICE pointers (e.g. from a torch
 *    tensor's data_ptr()).  Buffers are contiguous and row-major with a pitch
 *    equal to the width: image u8 [height][width], disparity u16
 *    [height][width].  The caller owns them.  `left` and `right` may alias;
 *    the output must not alias either input.
 *  - `stream` is a hipStream_t (NULL = the legacy default stream).  Compute
 *    calls only enqueue work and return; the result is ready when the stream
 *    reaches that point.
 *  - Disparities are integers in [0, max_disp) (in 1/16 pixel with
 *    SGM_SUBPIXEL); 0xFFFF marks a pixel that fails the left-right check.
 *  - Ties in the winner-take-all go to the smallest disparity.
 *  - Errors are reported as negative return codes (or NULL) before anything
 *    is enqueued; sgm_last_error() returns a message for the calling thread.
 *  - A context is not thread-safe; use one per host thread or serialize.
 */
#ifndef SGM_H
#define SGM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sgm_ctx sgm_ctx;
typedef void *sgm_stream_t; /* a hipStream_t */

enum {
    SGM_OK = 0,
    SGM_EINVAL = -1,    /* invalid argument or parameter combination */
    SGM_ENOMEM = -2,    /* device allocation failed or budget exceeded */
    SGM_EHIP = -3,      /* a HIP runtime call failed (no GPU, launch error) */
    SGM_EBUSY = -4,     /* server: request not admitted (no slot / memory) */
    SGM_ECANCELED = -5  /* server: request cancelled or failed */
};

enum {
    SGM_MEDIAN3 = 1u,     /* 3x3 median of the left (and right) disparity */
    SGM_LRCHECK = 2u,     /* left-right consistency check */
    SGM_CENSUS_CSCT = 4u, /* center-symmetric census (Eq. 1) instead of the
                             full-window census */
    SGM_GRAPH = 8u,       /* replay a captured HIP graph of the pipeline when
                             sgm_compute is called again with the same
                             buffers (not while stage timing is enabled) */
    SGM_LR_FULL = 16u,    /* with SGM_LRCHECK: the right disparity map of the
                             check comes from a second full SGM with the right
                             image as base (costs C_R(x, d) = Hamming distance
                             of the right word at x and the left word at
                             x + d, Cmax past the right border; the same path
                             directions; smallest minimising d), instead of
                             the diagonal minimum of the left SGM's sums.
                             Twice the cost and aggregation work; the
                             workspace grows (sgm_set_options may allocate). */
    SGM_SUBPIXEL = 32u,   /* left disparities in 1/16 pixel: q = 16 d + f at
                             the winner d, f = floor((16 (a - c) + den) /
                             (2 den)) with a, b, c = S(d-1), S(d), S(d+1) and
                             den = a + c - 2b (the parabola vertex rounded
                             half up; f = 0 if d = 0, d = D-1 or den = 0);
                             the median runs on q and the left-right check on
                             (q + 8) >> 4; the output holds q (0xFFFF still
                             marks a failed check) */
    SGM_ADAPTIVE_P2 = 64u /* the P2 of each aggregation step from p - r to p
                             is max(P1, floor(P2 / (1 + |I(p) - I(p - r)|)))
                             on the SGM's base image: smaller across
                             intensity edges (uses the cost-volume
                             aggregation) */
};

/* Checks a parameter set without touching the GPU.  Returns SGM_OK or
 * SGM_EINVAL (message in sgm_last_error).  Rules:
 *   1 <= width <= 16000, height >= 1; 1 <= max_disp <= 256; n_paths in {2, 4, 8};
 *   width * height * Dp <= 2^30 (Dp = max_disp rounded up to 64, 128 or 256);
 *   census_w, census_h odd and >= 1; the census fits 64 bits (full:
 *   w*h <= 64; CSCT: (w*h - 1)/2 <= 64); P1, P2 >= 0;
 *   n_paths * (Cmax + P2) <= 65535, where Cmax = w*h - 1 (full) or
 *   (w*h - 1)/2 (CSCT), so that summed costs fit in 16 bits (the bound
 *   L_r <= C + P2 follows from the last term of Eq. 3); with
 *   SGM_ADAPTIVE_P2 the bound uses max(P1, P2), the largest penalty a step
 *   can take.  Also P1 <= 65535, and unknown flag bits are rejected. */
int sgm_validate(int width, int height, int max_disp, int P1, int P2, int n_paths,
                 int census_w, int census_h, unsigned flags);

/* Creates a context for one image size and parameter set on the current HIP
 * device and allocates its device workspace (sgm_footprint_bytes).
 * P1, P2 are the penalties of Eq. 3 for disparity changes of one and of more
 * than one level.  The path set is: 2 = left-to-right and top-to-bottom
 * (Sec. 4); 4 = the four axial directions; 8 = axial plus diagonal.
 * The environment variable SGM_TUNE="lanes_h,lanes_v,bits" sets the initial
 * kernel shape of every new context (the arguments of sgm_set_tuning; a
 * malformed or rejected value is ignored, and reported when SGM_LOG >= 2).
 * Returns NULL on error (SGM_EINVAL / SGM_ENOMEM / SGM_EHIP). */
sgm_ctx *sgm_create(int width, int height, int max_disp, int P1, int P2, int n_paths,
                    int census_w, int census_h);

/* Options: SGM_MEDIAN3, SGM_LRCHECK, SGM_CENSUS_CSCT; lr_threshold is the
 * largest accepted |D_L(x) - D_R(x - D_L(x))| (default: flags 0, threshold 1).
 * Switching the census kind re-validates the overflow bound. */
int sgm_set_options(sgm_ctx *ctx, unsigned flags, int lr_threshold);

/* Enqueues the whole pipeline on `stream`: left u8 [H][W] is the base image,
 * right u8 [H][W] the match image (a left pixel x matches right pixel x - d,
 * Eq. 2); disp_out u16 [H][W] receives the disparity.  Asynchronous. */
int sgm_compute(sgm_ctx *ctx, const uint8_t *left, const uint8_t *right, uint16_t *disp_out,
                sgm_stream_t stream);

/* Kernel shapes (results never depend on them):
 *   lanes_h - lanes per horizontal aggregation slice (16, 32 or 64), lanes_v
 *   - lanes per vertical / diagonal slice (16 or 32), with lanes_h >= lanes_v
 *   (the shapes 16/16, 32/16, 32/32, 64/16 and 64/32; 64 acts as 32 when the
 *   padded range is 64 levels); 0 and 0 select the built-in default.
 *   fused   - bit SGM_TUNE_FUSED_AGG: the aggregation computes the matching
 *   costs from census words itself (no cost volume in memory); otherwise a
 *   cost kernel writes the u8 cost volume C[H][W][Dp] that the aggregation
 *   reads.  Bit SGM_TUNE_FUSED_CENSUS_COST (9x7 windows): that cost volume
 *   comes from one census + cost launch instead of a census launch and a cost
 *   launch.  Bit SGM_TUNE_FINAL_PASS: the last path direction (right-to-left;
 *   left-to-right with 2 paths) runs fused with the sum over directions and
 *   the winner-take-all (Sec. 3.3), so its L_r is never stored; used where
 *   the planes are u8, the cost volume is stored and neither SGM_LR_FULL
 *   nor SGM_ADAPTIVE_P2 is set, otherwise ignored.  Bit
 *   SGM_TUNE_POST_IN_WTA: the median (Sec. 2) and left-right check (Sec. 5) run
 *   inside the winner-take-all launch (the block that completes the raw rows
 *   around a row filters it) instead of a launch of their own; ignored with
 *   the final pass or without a post stage.  Default 0.
 * sgm_get_tuning reports the shape in effect. */
enum { SGM_TUNE_FUSED_AGG = 1, SGM_TUNE_FUSED_CENSUS_COST = 2, SGM_TUNE_FINAL_PASS = 4, SGM_TUNE_POST_IN_WTA = 8 };
int sgm_set_tuning(sgm_ctx *ctx, int lanes_h, int lanes_v, int fused);
int sgm_get_tuning(sgm_ctx *ctx, int *lanes_h, int *lanes_v, int *fused);

/* Releases the context and its workspace (synchronizes the device first).
 * NULL is accepted. */
void sgm_destroy(sgm_ctx *ctx);

/* Message of the last failed call on this thread ("" if none).  With the
 * environment variable SGM_LOG=1 every such message is also printed on
 * stderr when it is set; SGM_LOG=2 adds resource events (workspace growth,
 * graph captures). */
const char *sgm_last_error(void);

/* Device bytes a context of this shape needs (workspace only; the caller's
 * images and output are not counted).  0 if the shape is invalid. */
size_t sgm_footprint_bytes(int width, int height, int max_disp, int n_paths, unsigned flags);

/* ---- allocation-free computation ----
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the whole
 * pipeline of sgm_create + sgm_set_options + sgm_compute in one call that
 * allocates nothing.  The pair's workspace (sgm_footprint_bytes-like: cost
 * volume, L_r planes, census words, raw maps) lives in a static device array
 * of SGM_NOALLOC_MAX_BYTES bytes inside the library, which every GPU the
 * library runs on holds until the process ends.  A shape whose workspace
 * exceeds it returns SGM_ENOMEM (640x480, D = 128, 4 paths with u8 planes
 * needs 193 MiB; the full left-right check doubles the planes).  Arguments
 * are those of sgm_create and sgm_set_options (SGM_GRAPH is rejected) plus
 * the buffers of sgm_compute; the default kernel shapes are used.
 * Every call on a device shares that device's array and leaves its
 * contents behind (nothing needs clearing: each call writes every workspace
 * byte it reads): calls whose work overlaps on one device - on different
 * streams, or from different threads - race, so serialize them (one stream).
 * Asynchronous like sgm_compute. */
#define SGM_NOALLOC_MAX_BYTES ((size_t)256 << 20)
int sgm_compute_noalloc(int width, int height, int max_disp, int P1, int P2, int n_paths, int census_w,
                        int census_h, unsigned flags, int lr_threshold, const uint8_t *left,
                        const uint8_t *right, uint16_t *disp_out, sgm_stream_t stream);

/* ---- batches: many pairs of different shapes in one set of launches ----
 * One item is one stereo pair with its own size (w x h), disparity range,
 * path count and options; the census window and P1, P2 belong to the batch
 * (or server).  Buffers follow the conventions above.  Item flags:
 * SGM_MEDIAN3, SGM_LRCHECK, SGM_SUBPIXEL, SGM_LR_FULL (with SGM_LRCHECK),
 * SGM_ADAPTIVE_P2, SGM_CENSUS_CSCT, and the item's left-right threshold as
 * SGM_ITEM_LR_THRESHOLD(t), t in [0, 255]; without it the threshold is 1 (as
 * for sgm_set_options). */
typedef struct {
    int w, h, max_disp, n_paths;
    unsigned flags;
    const uint8_t *left;
    const uint8_t *right;
    uint16_t *out;
} sgm_item;

#define SGM_ITEM_THRESHOLD_SET 0x100u
#define SGM_ITEM_LR_THRESHOLD(t) (SGM_ITEM_THRESHOLD_SET | (((unsigned)(t) & 0xFFu) << 16))

typedef struct sgm_batch sgm_batch;

/* A batch runner on the current HIP device.  NULL on error. */
sgm_batch *sgm_batch_create(int P1, int P2, int census_w, int census_h);

/* Enqueues all n items on `stream`: one census, one cost, one aggregation,
 * one sum + winner-take-all and one median + LR launch for the whole batch
 * (items with SGM_LR_FULL add their right-base costs, directions and rows to
 * the same launches).
 * The aggregation is a persistent kernel whose wavefronts take (pair,
 * direction, slice group) work items, longest first, from a queue.  The
 * runner keeps a device workspace that grows to the largest batch seen;
 * growing it waits for the device to go idle first.  Items must not share
 * output buffers.  Results are identical to n separate sgm_compute calls. */
int sgm_batch_compute(sgm_batch *b, const sgm_item *items, int n, sgm_stream_t stream);

/* Kernel shape of the batched aggregation (results never depend on it):
 * lanes per horizontal slice (16 or 32) and per other slice (16 or 32) for
 * every pair; 0 keeps the per-pair default (32 horizontal lanes when the
 * image is wider than tall, else 16; 16 for the other directions). */
int sgm_batch_set_tuning(sgm_batch *b, int lanes_h, int lanes_v);

/* Workgroups (4 wavefronts each) of the persistent aggregation grid: 0, the
 * default, fills the device (512); 1 has one CU take the work items four at
 * a time, a check that no result depends on their order or concurrency
 * (results never depend on it). */
int sgm_batch_set_grid(sgm_batch *b, int max_workgroups);

/* Graph replay for batches (enable 1; 0, the default, launches directly).
 * With it on, sgm_batch_compute captures the batch's launches into a
 * hipGraph the first time it sees a batch signature (the runner's kernel
 * shape and every item's w, h, max_disp, n_paths and flags, in order) and
 * replays that graph for later batches with the same signature, whatever
 * their buffers: the graph's kernels read the items' pointers from a
 * descriptor table that belongs to the graph, copied again on `stream`
 * ahead of the replay when it changed.  Up to 8 graphs are kept, most
 * recently used first; capturing a new one waits for `stream`, and dropping
 * one (or turning graphs off) waits for the device.  Results are identical
 * to direct launches.  Calls on different streams must not overlap (a
 * replay and the next descriptor copy of the same graph are ordered by the
 * stream only). */
int sgm_batch_set_graph(sgm_batch *b, int enable);

/* Device bytes sgm_batch_compute needs for these items (0 if one is invalid). */
size_t sgm_batch_footprint(sgm_batch *b, const sgm_item *items, int n);

/* Releases the runner (synchronizes the device first).  NULL is accepted. */
void sgm_batch_destroy(sgm_batch *b);

/* One-shot convenience: create a runner, compute, wait for the stream,
 * destroy. */
int sgm_compute_batch(const sgm_item *items, int n, int P1, int P2, int census_w, int census_h,
                      sgm_stream_t stream);

/* ---- request server: continuous batching on one device ----
 * A server owns a device workspace of a fixed byte budget (allocated once,
 * kept resident), `max_slots` launch slots over `n_streams` streams and a
 * scheduler thread.  Requests (one stereo pair each, an sgm_item) may be
 * submitted from any host thread at any time.  Whenever a slot is free, the
 * scheduler takes queued requests in arrival order for as long as their
 * workspaces fit in the free part of the budget (admission by HBM footprint;
 * first fit) and launches them as one group (a group of one through the
 * single-pair kernels, larger groups through the batched kernels).  Slots
 * sharing a stream run their groups back to back without waiting for the
 * host; slots on different streams run concurrently.  Requests arriving while
 * groups run join the next group.  A result is identical to sgm_compute's
 * for the same pair, whatever else ran beside it.  While groups are in flight
 * the scheduler thread polls their completion events (it keeps one host core
 * busy).
 *
 * The caller's images and output of a request must stay valid and untouched
 * until the request reaches a final state.  No call may use a server during
 * or after sgm_server_destroy. */
typedef struct sgm_server sgm_server;

enum {
    SGM_REQ_QUEUED = 0,   /* waiting for a stream and workspace */
    SGM_REQ_RUNNING = 1,  /* launched; results not yet complete */
    SGM_REQ_DONE = 2,     /* output written */
    SGM_REQ_CANCELED = 3, /* removed before it started */
    SGM_REQ_FAILED = 4    /* a launch or the device failed */
};

typedef struct {
    uint64_t submitted, completed, rejected, canceled, failed;
    uint64_t groups;           /* launch groups started */
    uint64_t grouped_requests; /* requests over all groups (mean group size =
                                  grouped_requests / groups) */
    uint64_t pending, running; /* current queue length, requests in flight */
    size_t bytes_in_use, peak_bytes, budget_bytes;
    uint64_t timed_out;        /* requests failed by the watchdog (also in failed) */
    uint64_t draining_groups;  /* stuck groups the device has not completed yet */
} sgm_server_stats;

/* Creates a server on the current HIP device.  hbm_budget_bytes: workspace
 * bytes to reserve (rounded down to 256); max_slots in [1, 16]: groups in
 * flight at once, each slot on a stream of its own (slots on different
 * streams run concurrently); P1, P2 and the census window apply to every
 * request.  NULL on error (SGM_EINVAL for bad parameters, SGM_ENOMEM if the
 * budget cannot be allocated). */
sgm_server *sgm_server_create(size_t hbm_budget_bytes, int max_slots, int P1, int P2, int census_w,
                              int census_h);

/* As sgm_server_create, with the slots spread round-robin over n_streams
 * streams, n_streams in [1, max_slots] (1 = groups run one after another in
 * admission order; slots sharing a stream run their groups back to back
 * without waiting for the host). */
sgm_server *sgm_server_create_ex(size_t hbm_budget_bytes, int max_slots, int n_streams, int P1, int P2,
                                 int census_w, int census_h);

/* Group limits, queue length and overlap.  A group takes at most max_group
 * requests (default 32, at most 256) and, unless it holds a single request,
 * at most max_group_cells cells in total (W * H * max_disp * n_paths summed
 * over its requests; default 2^28): requests that fill the device alone run
 * alone (grouping them measured slower), small ones run in groups (faster
 * once the requests' launches outpace the device).  The queue accepts at most max_pending requests (default 4096).
 * While a group runs, a second one starts beside it only when at least
 * overlap_queue requests are queued (default 3; 1 = whenever a slot is
 * free): at light load a request waits for the running one rather than
 * sharing the device with it. */
int sgm_server_set_policy(sgm_server *s, int max_group, int max_pending, uint64_t max_group_cells,
                          int overlap_queue);

/* Watchdog on completion events: a group still running timeout_ms after
 * its launch is declared stuck, and its requests end as SGM_REQ_FAILED at
 * once (counted in stats.timed_out), so that their callers stop waiting.
 * The device work cannot be taken back: the group's workspace and slot stay
 * reserved until its completion event fires (stats.draining_groups counts
 * such groups), and until then the device may still read the requests'
 * images and write their outputs, so a caller must not reuse those buffers
 * before draining_groups is back to 0.  0 (the default) turns it off. */
int sgm_server_set_watchdog(sgm_server *s, int timeout_ms);

/* Workspace bytes a request takes from the budget (0 if invalid). */
size_t sgm_server_request_bytes(sgm_server *s, const sgm_item *req);

/* Queues one request and returns its ticket.  SGM_EINVAL: invalid request
 * (checked here, before queueing); SGM_ENOMEM: its workspace alone exceeds
 * the budget, so it could never be admitted; SGM_EBUSY: the queue is full
 * (the request is rejected, not queued). */
int sgm_server_submit(sgm_server *s, const sgm_item *req, uint64_t *ticket);

/* State of a request (SGM_REQ_*) and, once final, its latency in seconds
 * from submission to completion.  A ticket is retired once a call has
 * reported a final state; using it again gives SGM_EINVAL. */
int sgm_server_poll(sgm_server *s, uint64_t ticket, int *status, double *latency_s);

/* As sgm_server_poll, after waiting up to timeout_ms (< 0: no limit) for a
 * final state. */
int sgm_server_wait(sgm_server *s, uint64_t ticket, int timeout_ms, int *status, double *latency_s);

/* Cancels a request that has not started (SGM_EBUSY if it has). */
int sgm_server_cancel(sgm_server *s, uint64_t ticket);

int sgm_server_get_stats(sgm_server *s, sgm_server_stats *out);

/* Cancels queued requests, waits for running groups to complete, then frees
 * everything.  NULL is accepted. */
void sgm_server_destroy(sgm_server *s);

/* ---- stage timing ----
 * sgm_profile_enable(ctx, n) with n > 0 makes every n-th sgm_compute record
 * HIP events on its stream before the first stage and after each of the four
 * stages (0 census + cost, 1 aggregation, 2 sum + winner-take-all, 3 median +
 * LR); n = 0 turns timing off.  sgm_profile_read waits for the recorded
 * calls, writes the summed milliseconds of each stage into stage_ms[4] and the
 * number of recorded calls into *ncalls, and clears them. */
int sgm_profile_enable(sgm_ctx *ctx, int every_n);
int sgm_profile_read(sgm_ctx *ctx, double *stage_ms, int *ncalls);

/* Allocation-failure hook, for tests of failure handling (process-wide,
 * any thread): the next `after` device or pinned host allocations the
 * library makes succeed and the `count` after them fail as if the memory
 * were exhausted, so the call that needed them returns SGM_ENOMEM (a
 * server request fails with SGM_REQ_FAILED) and no kernel is launched for
 * it.  sgm_debug_fail_alloc(0, 0) turns it off. */
void sgm_debug_fail_alloc(int after, int count);

/* ---- debug taps: intermediates for stage-by-stage parity tests ---- */

/* Census words of one image: u64 [H][W] (CSCT words use the low bits). */
int sgm_debug_census(sgm_ctx *ctx, const uint8_t *img, uint64_t *census_out,
                     sgm_stream_t stream);

/* Runs the pipeline up to the summed costs and writes S u16 [H][W][max_disp]
 * (d fastest), S(p, d) = sum over directions of L_r(p, d). */
int sgm_debug_sums(sgm_ctx *ctx, const uint8_t *left, const uint8_t *right, uint16_t *s_out,
                   sgm_stream_t stream);

/* Partial sums of the aggregation schedule, u16 [H][W][max_disp] (d
 * fastest).  The last direction of the path set (right-to-left; with 2 paths
 * left-to-right) is the one the final pass fuses with the sum and the
 * winner-take-all (Sec. 3.3), so the schedule has two phases:
 *   phase 0: S_0(p, d) = sum of L_r(p, d) over every other direction (the
 *            planes the first aggregation launch stores);
 *   phase 1: S(p, d) = S_0(p, d) + L_last(p, d), the sums the final pass
 *            takes its winners from (Eq. 4).
 * Other phases return SGM_EINVAL. */
int sgm_debug_phase_sums(sgm_ctx *ctx, const uint8_t *left, const uint8_t *right, int phase,
                         uint16_t *s_out, sgm_stream_t stream);

/* One intermediate as u16 [H][W][max_disp] (d fastest): which = -1 gives the
 * matching cost C (Eq. 2); which = r in [0, n_paths) gives L_r of path
 * direction r (Eq. 3), directions numbered as for sgm_create: (1,0), (-1,0),
 * (0,1), (0,-1), (1,1), (-1,1), (1,-1), (-1,-1); with 2 paths (1,0), (0,1).
 * With SGM_LR_FULL, which = -2 gives the right-base costs C_R and which =
 * n_paths + r the right-base L_r of direction r. */
int sgm_debug_stage(sgm_ctx *ctx, const uint8_t *left, const uint8_t *right, int which,
                    uint16_t *out, sgm_stream_t stream);

/* Raw (before median / LR) left and right disparity maps, u16 [H][W] each. */
int sgm_debug_raw_disparity(sgm_ctx *ctx, const uint8_t *left, const uint8_t *right,
                            uint16_t *dl_out, uint16_t *dr_out, sgm_stream_t stream);

/* Measurement helper: VALU rates the aggregation's arithmetic (Eq. 3 on u16
 * pairs, its DPP and permlane group minimum) is compared with.  Enqueues
 * `blocks` blocks of 256 threads; time them with events on `stream`.
 *   mode 0: throughput - each lane runs `iters` rounds of 8 independent
 *           packed add + packed min pairs (16 VALU instructions per wave per
 *           round);
 *   mode 1..3: latency - one dependent chain per lane, 8 links per round:
 *           1 packed add then packed min, 2 a minimum with a DPP row_mirror
 *           operand then an add, 3 a permlane16 swap, a minimum and an add.
 * sink: device u32 [blocks * 256], written only in a case that does not
 * occur (it keeps the work).  SGM_EINVAL for a mode outside 0 .. 3, blocks
 * outside [1, 2^20], iters < 1 or a null sink. */
int sgm_debug_valu_probe(int mode, int blocks, int iters, uint32_t *sink, sgm_stream_t stream);

/* Host-only: the pixels a GPU aggregation slice visits.  Direction
 * (rx, ry) in {-1,0,1}^2 \ {(0,0)}; slice in [0, number of slices) where
 * horizontal directions have H slices of W steps and the others W slices of H
 * steps.  Diagonal slices wrap from one side border to the other and restart
 * the path there (Sec. 3.2).  Writes up to max_steps (x, y, restart) triples;
 * restart = 1 where the step begins a new path.  Returns the step count or
 * SGM_EINVAL. */
int sgm_path_walk(int width, int height, int rx, int ry, int slice, int max_steps, int *xs,
                  int *ys, uint8_t *restart);

#ifdef __cplusplus
}
#endif

#endif /* SGM_H */
