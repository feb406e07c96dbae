/*
 * lk_serve.h -- a serving loop on top of the LightKernel dispatch library: requests
 * (uneven work items) arrive over time, are admitted against a device-memory budget and
 * executed by the persistent workers with continuous batching.
 *
 * The paper motivates persistent threads with handing work to chosen clusters at run
 * time with little overhead (Sec. 1, Sec. 2.3) and names finer-grained kernels as what a
 * light Trigger enables (Sec. 3); this is that use: many small and large requests kept
 * in flight together on one GPU.
 *
 * Model.  Every request reads resident device buffers (its inputs are addresses inside
 * buffers that stay on the device for the whole run) and, if it produces an array, gets
 * an output buffer carved from a caller-provided device arena whose size is the memory
 * budget.  A request is admitted when it has arrived and its output fits; admission is
 * first come, first served (a request that does not fit waits, and so do those behind
 * it).  An admitted request is cut into tiles of tile_elems elements; tiles of all
 * admitted requests are queued in admission order and posted to free mailbox slots,
 * breadth first (every idle worker gets a tile before any worker gets a second), so work
 * from requests that arrived while others are running overlaps with theirs on the GPU and
 * does not queue behind it while a worker is idle.  When its last tile completes the request is done, its int64 result is the exact
 * sum of its tiles' partial results, and its output memory returns to the budget (unless
 * `retain` is set).
 *
 * Host threads.  `threads` scheduler threads each own the workers w with w % threads ==
 * s, the requests r with r % threads == s and an equal slice of the arena (one producer
 * per mailbox, no locks on the dispatch path).  A request's tiles run only on its own
 * scheduler's workers, so fewer schedulers let a large request spread over more CUs,
 * while each scheduler must keep up with its share of the tile rate: on 256 CUs, 3-4
 * schedulers gave the lowest latencies from 10 k to 1 M requests/s, one fell behind
 * at 1 M/s and 14 left the largest requests on 18 workers.
 */
#ifndef LK_SERVE_H
#define LK_SERVE_H

#include <stdint.h>

#include "lk.h"

#ifdef __cplusplus
extern "C" {
#endif

/* One request (48 bytes). */
typedef struct lks_request {
  double arrival_us;  /* arrival time, microseconds after the start of the run */
  uint32_t op;        /* LK_OP_AFFINE_SUM_I32, LK_OP_SUM_I32_I64, LK_OP_AXPY_F32 or LK_OP_COPY_F32 */
  int32_t a, b;       /* AFFINE_SUM_I32 coefficients */
  float alpha;        /* AXPY_F32 */
  uint64_t n;         /* elements */
  uint64_t in;        /* device address of the input (x) */
  uint64_t in2;       /* AXPY_F32: device address of y; 0 otherwise */
} lks_request;

typedef struct lks_config {
  uint64_t arena;       /* device address of the output arena (256-byte aligned) */
  uint64_t arena_bytes; /* its size: the device-memory budget for request outputs */
  uint64_t tile_elems;  /* elements per tile, a positive multiple of 256 */
  uint32_t threads;     /* scheduler threads, 1..64, at most the number of workers */
  uint32_t retain;      /* 1: never recycle output memory (all outputs stay readable) */
  int64_t timeout_ns;   /* a tile not finished this long after posting fails the run */
} lks_config;

/* Outcome of one request (40 bytes). */
typedef struct lks_outcome {
  int64_t result;       /* exact int64 result (AFFINE_SUM_I32, SUM_I32_I64), else 0 */
  uint64_t out;         /* device address of its output (valid while retained), or 0 */
  double admit_us;      /* admission time (same clock as arrival_us) */
  double done_us;       /* completion observed */
  int32_t status;       /* LK_OK, or the error that stopped the run before it finished */
  uint32_t tiles;       /* tiles it was cut into */
} lks_outcome;

typedef struct lks_stats {
  double elapsed_s;       /* first arrival to last completion */
  uint64_t tiles;         /* tiles whose completion the schedulers took */
  uint64_t deferred;      /* admissions that had to wait for memory */
  uint64_t peak_bytes;    /* peak output memory in use, summed over shards */
  uint64_t posted;        /* tiles posted */
  uint64_t drained;       /* tiles waited for after an error stopped the run (posted =
                             tiles + drained whenever lks_run returns with the context
                             still running) */
} lks_stats;

/* Serve `count` requests on a running context whose clusters are one worker each
 * (LK_CLUSTERS_PER_WORKER).  Requests must be sorted by arrival time.  Fills out[i] for
 * every request and *stats.  Errors: LK_EINVAL (bad arguments, a request that can never
 * fit its shard's budget, or -- with retain -- a budget exhausted for good), errors of
 * lk_submit / lk_wait, LK_ETIMEDOUT.
 * When a scheduler stops on an error, every scheduler stops and first waits for the tiles
 * it has posted (each for max(timeout_ns, 1 s), or without a deadline when timeout_ns < 0),
 * so that on return no tile of the run still reads or writes memory.  If a tile does not
 * finish in that time, lks_run disposes the context (lk_dispose) before returning: either
 * the workers end, or the context is left poisoned (lk_get_info state 2), in which case the
 * arena and the request buffers may still be written by the GPU and must stay allocated. */
LK_API int lks_run(lk_ctx *ctx, const lks_config *cfg, const lks_request *reqs, uint64_t count,
                   lks_outcome *out, lks_stats *stats);

#ifdef __cplusplus
}
#endif
#endif /* LK_SERVE_H */
