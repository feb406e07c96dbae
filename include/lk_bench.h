/*
 * lk_bench.h -- native timed runners, per-launch baselines and roofline probes of the
 * LightKernel library (same shared library as lk.h).
 *
 * The paper measures host-side time per phase (Sec. 3, Tables 2-3) for its persistent
 * path and for "traditional" kernels (Alloc, Launch, Wait, Dispose).  These runners take
 * the same measurements in native code, so that no interpreter overhead sits inside a
 * timed region:
 *   - lkb_serial        Trigger + Wait per item on a running context, item after item;
 *   - lkb_lanes         many clusters fed back-to-back by host threads;
 *   - lkb_isolation     a periodic critical item on one cluster beside streaming
 *                       interference on the others;
 *   - lkb_batch         bursts of uneven items as one batch over a cluster;
 *   - lkb_launch_burst  the same bursts as per-item launches or a captured hipGraph;
 *   - lkb_replay        the paper's phase protocol (Init/Trigger/Wait/Dispose vs
 *                       Alloc/Spawn/Wait/Dispose) with its compute-only item;
 *   - lkb_launch_serial one ordinary kernel launch per item (the paper's spawn path),
 *                       optionally through a single-node hipGraph relaunched per item;
 *                       lkb_launch_serial_static is its form that allocates nothing;
 *   - lkb_launch_lanes  the lanes workload with one launch (or graph launch) per item;
 *   - lkb_pingpong      the bare host<->device echo: the floor of any mailbox round trip;
 *   - lkb_copy          streaming-copy bandwidth: the HBM roofline, and the known-size
 *                       kernel used to scale memory-traffic counters.
 * Latencies are host steady-clock microseconds.  All pointers in lkb_item are device
 * addresses owned by the caller.  Every function returns LK_OK or a negative LK_E* code.
 */
#ifndef LK_BENCH_H
#define LK_BENCH_H

#include <stdint.h>

#include "lk.h"

#ifdef __cplusplus
extern "C" {
#endif

/* One work item with its in/out references (56 bytes). */
typedef struct lkb_item {
  uint32_t op;      /* LK_OP_* */
  int32_t a, b;     /* AFFINE_SUM_I32 coefficients; SPIN: a = iterations */
  float alpha;      /* SAXPY_F32 / AXPY_F32 */
  uint64_t n;       /* elements */
  uint64_t in, out; /* device addresses */
  uint64_t in2;     /* AXPY_F32: device address of y; 0 otherwise */
  uint32_t flags;   /* LK_DF_* descriptor flags: honoured by the persistent paths, ignored
                       by the per-launch ones (a launched kernel keeps nothing across items) */
  uint32_t reserved;
} lkb_item;

/* Submit-then-wait each item on `cluster` in order (the paper's Trigger then Wait).
 * results[i] = the item's int64 result; lat_us[i] = lk_submit start to lk_wait return;
 * trigger_us[i] = duration of lk_submit alone; info (nullable) = device-side timing.
 * Any of the output arrays may be NULL.  Stops at the first error and returns it. */
LK_API int lkb_serial(lk_ctx *c, uint32_t cluster, const lkb_item *items, uint64_t count, int64_t timeout_ns,
               int64_t *results, double *lat_us, double *trigger_us, lk_completion *info);

/* Feed n_lanes clusters back-to-back: lane l posts items[l*items_per_lane + k] to
 * lane_cluster[l] in order, keeping up to `in_flight` of them posted, and is served by
 * host thread l % n_threads.  lat_us[l*items_per_lane + k] = submit to completion
 * observed; results and info (device-side timing) likewise, each nullable;
 * *elapsed_s = first submit to last completion. */
LK_API int lkb_lanes(lk_ctx *c, const uint32_t *lane_cluster, uint32_t n_lanes, const lkb_item *items,
              uint64_t items_per_lane, uint32_t in_flight, uint32_t n_threads, int64_t timeout_ns,
              int64_t *results, double *lat_us, double *elapsed_s, lk_completion *info);

/* Cluster isolation: a critical item is released on crit_cluster every period_ns (host
 * busy-wait to t0 + k * period, item k = crit[k]), submitted and waited for, while each
 * cluster bg_clusters[i] runs bg[i] back-to-back from its own host thread (re-posted as
 * soon as it completes).  Per period: lat_us = release to lk_wait return, late_us =
 * release to submit (host lateness), results and info (device-side timing); bg_done[i] =
 * background items completed; *elapsed_s = run time.  The calling thread is pinned to
 * the last host core for the run and background threads to the others. */
LK_API int lkb_isolation(lk_ctx *c, uint32_t crit_cluster, const lkb_item *crit, uint64_t periods, int64_t period_ns,
                  const uint32_t *bg_clusters, uint32_t n_bg, const lkb_item *bg, int64_t *results, double *lat_us,
                  double *late_us, lk_completion *info, uint64_t *bg_done, double *elapsed_s);

/* The paper's evaluation protocol (Sec. 3, Tables 2-3) on this hardware: `runs` times,
 * (1) persistent path: Init (lk_init with n_workers workers in one cluster), Trigger
 * (lk_submit of one SPIN item of spin_iters iterations per thread, one slice per
 * worker), Wait (lk_wait), Dispose (lk_dispose);
 * (2) per-launch path: Alloc (hipMalloc + stream creation), Spawn (launch of the same
 * SPIN item on n_workers workgroups), Wait (stream synchronisation), Dispose (stream
 * destruction + hipFree).
 * Phase r*4 + {0,1,2,3} of each output: microseconds (lk_us, hip_us) and host
 * time-stamp-counter cycles (lk_cycles, hip_cycles); results[2r] and results[2r + 1]
 * receive run r's item result on the persistent and on the per-launch path (the sum over
 * its workers / workgroups; the compute-only item's result is 0), read outside the timed
 * phases; any output may be NULL. */
LK_API int lkb_replay(int device, uint32_t n_workers, uint32_t spin_iters, uint32_t runs, double *lk_us,
               double *hip_us, uint64_t *lk_cycles, uint64_t *hip_cycles, int64_t *results);

/* Batches: `reps` times, post one batch of n_tiles device tiles to `cluster` and wait for
 * it; makespan_us[r] = lk_submit_batch start to lk_wait return; info (nullable) = the
 * members' device-side timing.  LK_EFAULT if a batch did not execute exactly n_tiles. */
LK_API int lkb_batch(lk_ctx *c, uint32_t cluster, const lk_tile *tiles, uint32_t n_tiles, int64_t *partials,
              uint32_t reps, int64_t timeout_ns, double *makespan_us, lk_completion *info);

/* The same items as ordinary launches: one launch per item on one stream (grid =
 * ceil(n / elems_per_wg) workgroups, at most 4096) then one stream synchronisation, or,
 * with mode LKB_USE_GRAPH, the launches captured once into a hipGraph (capture and
 * instantiation not timed) and the graph launched.  makespan_us[r] per repetition. */
LK_API int lkb_launch_burst(int device, const lkb_item *items, uint32_t count, uint64_t elems_per_wg,
                     uint32_t threads, uint32_t mode, uint32_t reps, double *makespan_us);

#define LKB_COMPLETE_SYNC 0u  /* completion observed by hipStreamSynchronize */
#define LKB_COMPLETE_FLAG 1u  /* completion observed through a host-coherent word the
                                 kernel's last workgroup writes (system-scope release) */
#define LKB_USE_GRAPH 2u      /* launch through a single-node hipGraph whose kernel node
                                 parameters are updated per item */
#define LKB_GRAPH_CHAIN 4u     /* lkb_launch_lanes: one captured chain of kernel nodes per lane */

/* One launch per item on one stream, grid = k workgroups of `threads` (slice j per
 * workgroup, the same slicing rule and op bodies as the persistent path).
 * mode = LKB_COMPLETE_SYNC or LKB_COMPLETE_FLAG, optionally | LKB_USE_GRAPH.
 * lat_us[i] = launch start to completion observed; launch_us[i] = the launch call. */
LK_API int lkb_launch_serial(int device, uint32_t k, uint32_t threads, const lkb_item *items, uint64_t count,
                      uint32_t mode, int64_t *results, double *lat_us, double *launch_us);

/* Allocation-free form of lkb_launch_serial with mode LKB_COMPLETE_SYNC, for callers that
 * cannot allocate (loops or harnesses in which hipMalloc, hipHostMalloc and stream
 * creation are not allowed).  Same items, grid, slicing, results and timings; instead of
 * a stream and a host-coherent partial-result array created per call, the launches go to
 * the null stream and the k per-workgroup partials go to a static device array of the
 * library (32 KiB per GPU, held until the process ends), read back with hipMemcpy after
 * each item's stream synchronisation (outside lat_us).  k is limited to 1..4096
 * (LK_EINVAL beyond, with nothing launched).  Every call on one GPU shares that GPU's
 * array: calls that overlap in time on the same GPU, from any threads, race on it and
 * their results are undefined. */
LK_API int lkb_launch_serial_static(int device, uint32_t k, uint32_t threads, const lkb_item *items,
                                    uint64_t count, int64_t *results, double *lat_us, double *launch_us);

/* The lanes workload with one launch per item: lane l runs on stream l % n_streams, one
 * item in flight per lane, completion observed through the flag form, host thread
 * l % n_threads.  mode = 0 or LKB_USE_GRAPH.  Outputs as lkb_lanes.
 * mode = LKB_GRAPH_CHAIN instead captures each lane's items once as one hipGraph, a chain
 * of items_per_lane kernel nodes (capture and instantiation not timed), then times the
 * launch of every lane's graph on stream l % n_streams until all streams are idle: the
 * throughput form of the graph baseline.  results[] are filled; no per-item completion is
 * observed, so lat_us[] entries are set to 0 and *elapsed_s covers the whole run. */
LK_API int lkb_launch_lanes(int device, uint32_t n_lanes, const lkb_item *items, uint64_t items_per_lane,
                     uint32_t n_streams, uint32_t n_threads, uint32_t threads, uint32_t mode,
                     int64_t *results, double *lat_us, double *elapsed_s);

/* Host<->device echo over fine-grained host-coherent memory: `workers` one-wave
 * workgroups (one per CU when spread != 0) each echo `iters` values; the host thread
 * writes value v to worker w's word and waits for the echo, workers in turn.
 * rtt_us[w*iters + i] receives each round trip (NULL allowed). */
LK_API int lkb_pingpong(int device, uint32_t workers, uint64_t iters, uint32_t poll_sleep, int spread,
                 double *rtt_us);

/* Streaming copy of `bytes` (multiple of 16, 16-byte aligned device buffers) with `grid`
 * workgroups of `threads` (64..1024, whole waves), each thread keeping `unroll` (4, 8 or
 * 16) 16-byte vectors in flight, repeated `reps` times after one untimed copy; *ms_avg =
 * average kernel time from HIP events; *gbps = 2*bytes / time (read + write).  policy:
 * LKB_COPY_PLAIN ordinary loads and stores, LKB_COPY_NONTEMPORAL non-temporal loads and
 * stores, LKB_COPY_SYSTEM ordinary loads and stores written through the L2 (cache
 * policy sc0 sc1, the persistent worker's output path; bytes below 2 GiB). */
#define LKB_COPY_PLAIN 0u
#define LKB_COPY_NONTEMPORAL 1u
#define LKB_COPY_SYSTEM 2u
LK_API int lkb_copy(int device, const void *src, void *dst, uint64_t bytes, uint32_t grid, uint32_t threads,
                    uint32_t unroll, uint32_t policy, uint32_t reps, double *ms_avg, double *gbps);

#ifdef __cplusplus
}
#endif
#endif /* LK_BENCH_H */
