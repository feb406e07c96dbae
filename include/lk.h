/*
 * lk.h -- C ABI of the LightKernel persistent-thread dispatch library for AMD Instinct
 * MI355X (gfx950).
 *
 * The method (paper Sec. 1, Sec. 2.3, Sec. 2.4): one persistent kernel is launched at
 * boot with exactly one workgroup ("worker") per compute unit (up to four per CU on
 * request, and optionally only on some XCDs: lk_config).  Each worker owns a pair
 * of mailboxes: to_GPU, where the host posts a command, and from_GPU, where the worker
 * reports its status (Sec. 2.4, Fig. 2, Table 1).  A command carries a descriptor of the
 * work plus references to its input and output data (Sec. 1).  Workers are grouped into
 * clusters, and a work item is submitted to one cluster (Sec. 1 and Sec. 2.1: work and
 * data are mapped onto a specific cluster to limit interference).  The host-side phases
 * follow Sec. 3: Init (lk_init), Trigger (lk_submit), Wait (lk_wait), Dispose
 * (lk_dispose).
 *
 * Conventions shared by every call:
 *   - every function returns an int: LK_OK (0) or a negative LK_E* code; nothing aborts,
 *     throws or exits;
 *   - device pointers are plain addresses in the calling process (for example a PyTorch
 *     tensor's data_ptr()); the caller owns them;
 *   - lk_strerror() names a code, lk_last_error() gives the calling thread's last detail.
 *
 * The persistent kernel is dispatched on an HSA queue of its own, outside every HIP
 * stream, so HIP and PyTorch work (default stream included) keeps running beside it on
 * the CUs the workers leave free.  The workers hold about 96 KiB of LDS on every CU they
 * occupy, which limits how much LDS other kernels can use there until lk_dispose.
 */
#ifndef LK_H
#define LK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Exported symbols of the shared library (it is built with hidden default visibility). */
#define LK_API __attribute__((visibility("default")))

/* ------------------------------------------------------------------ limits */
#define LK_MAX_WORKERS 1024u   /* workers per context (MI355X has 256 CUs) */
#define LK_MAX_DEPTH 64u       /* ring slots per mailbox; 1 is the paper's single slot */
#define LK_MAX_WORKERS_PER_CU 4u /* persistent workgroups resident on one CU */
#define LK_MAX_N (1ull << 40)  /* elements per work item */

/* ------------------------------------------------------------------ error codes */
enum {
  LK_OK = 0,
  LK_EINVAL = -1,     /* bad argument: null/misaligned pointer, unknown op, bad cluster... */
  LK_EAGAIN = -2,     /* lk_submit: a member mailbox has no free ring slot; nothing posted */
  LK_ETIMEDOUT = -3,  /* deadline passed; the ticket (or context) stays valid */
  LK_ESTATE = -4,     /* call not valid in the context's state (disposed, workers exited) */
  LK_ENODEV = -5,     /* no usable GPU, or the workers did not become resident */
  LK_EHIP = -6,       /* a HIP runtime call failed; lk_last_error() has its message */
  LK_EFAULT = -7      /* a worker rejected a descriptor (status ERROR) */
};

/* ------------------------------------------------------------------ work items
 * The paper's only work item is a compute-only loop (Sec. 3).  The item bodies below are
 * the evaluation workloads' items; n counts elements of the whole item.
 *
 *  LK_OP_NOP            no memory effect; result 0.
 *  LK_OP_AFFINE_SUM_I32 in = x (int32[n]), out = y (int32[n]):
 *                       y[i] = (a*x[i] + b) mod 2^32 read as two's complement;
 *                       result = sum over i of (int64)y[i] (exact).
 *  LK_OP_SUM_I32_I64    in = x (int32[n]), out unused (may be NULL);
 *                       result = sum over i of (int64)x[i] (exact).
 *  LK_OP_SAXPY_F32      in = x (float[n]), out = y (float[n]), in place:
 *                       y[i] = fmaf(alpha, x[i], y[i]), one binary32 fused multiply-add,
 *                       round to nearest even, subnormals preserved.
 *  LK_OP_COPY_F32       out[i] = in[i], bit for bit (float[n]).
 *  LK_OP_SPIN           compute-only loop of a iterations per thread (the paper's
 *                       benchmark item, Sec. 3); no memory effect; result 0.
 *  LK_OP_BATCH          many items in one dispatch: submitted only through
 *                       lk_submit_batch (see "batches" below).
 *  LK_OP_AXPY_F32       in = x (float[n]), aux = y (float[n], device address), out = result
 *                       (float[n]): out[i] = fmaf(alpha, x[i], y[i]); x and y are only read
 *                       (the out-of-place form of SAXPY, for inputs shared between items).
 */
enum {
  LK_OP_NOP = 0,
  LK_OP_AFFINE_SUM_I32 = 1,
  LK_OP_SUM_I32_I64 = 2,
  LK_OP_SAXPY_F32 = 3,
  LK_OP_COPY_F32 = 4,
  LK_OP_SPIN = 5,
  LK_OP_BATCH = 6,
  LK_OP_AXPY_F32 = 7,
  LK_OP_COUNT = 8
};

/* Descriptor of one work item, copied by value at submission (Sec. 1: "a descriptor of
 * the work").  The in/out references are passed beside it to lk_submit. */
typedef struct lk_desc {
  uint32_t op;        /* LK_OP_* */
  uint32_t flags;     /* LK_DF_*; 0 for plain items */
  uint64_t n;         /* element count, 0 .. LK_MAX_N; 0 is a valid no-op with result 0 */
  int32_t a, b;       /* AFFINE_SUM_I32 coefficients; SPIN: a = iterations */
  float alpha;        /* SAXPY_F32 coefficient */
  uint32_t reserved;  /* must be 0 */
  uint64_t aux;       /* AFFINE_SUM_I32 / SUM_I32_I64: optional device int64* with one entry
                         per cluster member (member j writes its partial result to aux[j]),
                         0 = none; AXPY_F32: the device address of y (required) */
  uint64_t user_tag;  /* opaque to the library; not interpreted */
} lk_desc;

/* Descriptor flags: keep x (the `in` operand) of a SAXPY_F32, AXPY_F32, AFFINE_SUM_I32 or
 * SUM_I32_I64 item in each member worker's local data share (LDS) across items, mapping
 * that operand onto the cluster that computes with it (Sec. 2.1: clusters are exposed so
 * that data, as well as work, can be placed on them, and their local memories keep data
 * next to the computation).
 *
 *  LK_DF_PIN_INPUT   a member holding a pinned slice with the same address and length
 *                    reads x from LDS instead of memory; otherwise it reads x from memory
 *                    and keeps it.  By setting the flag the caller promises that those
 *                    bytes are unchanged since the member pinned them.
 *  LK_DF_PIN_RELOAD  as LK_DF_PIN_INPUT, but always reads x from memory and replaces the
 *                    pinned copy: use it on the first item after x has changed.
 *
 * Each worker keeps up to 4 pinned slices (their raw 32-bit words, whatever the op), placed
 * one after another in its LDS: a new slice goes after the others while fewer than 4 are
 * held and all fit in lk_info.pin_capacity, otherwise it replaces all of them.  Items
 * without these flags leave the slices in place.  lk_submit rejects a flagged item (LK_EINVAL)
 * unless: the op is one of the four above; in, the out it writes (not SUM_I32_I64's) and
 * (AXPY_F32) y are 16-byte aligned; and every member's slice is a multiple of 4 elements
 * of at most lk_info.pin_capacity bytes.  n = 0 is accepted and pins
 * nothing.  Batches take no flags. */
#define LK_DF_PIN_INPUT  0x1u
#define LK_DF_PIN_RELOAD 0x2u

/* ------------------------------------------------------------------ clusters
 * Workers are numbered 0..n_workers-1 in physical order (XCD, shader engine, shader
 * array, CU), learnt at boot from each workgroup's hardware-id registers.
 *
 *  LK_CLUSTERS_PER_WORKER  cluster i = { worker i }
 *  LK_CLUSTERS_PER_XCD     cluster j = the workers on the j-th XCD present, in
 *                          ascending XCD order (8 clusters of 32 on a full MI355X)
 *  LK_CLUSTERS_ONE         one cluster holding every worker
 *  LK_CLUSTERS_EXPLICIT    cluster_of_worker[w] gives worker w's cluster; clusters are
 *                          numbered 0..n_clusters-1 and none may be empty
 *
 * An item submitted to a cluster of k members is split into k contiguous slices; slice j
 * goes to member j (ascending worker order) and covers [min(n, j*m), min(n, (j+1)*m))
 * with m = ceil(n/k) rounded up to a multiple of 256 elements.  Trailing slices may be
 * empty; every member still receives (and acknowledges) its slice.
 */
enum { LK_CLUSTERS_PER_WORKER = 0, LK_CLUSTERS_PER_XCD = 1, LK_CLUSTERS_ONE = 2,
       LK_CLUSTERS_EXPLICIT = 3 };

/* config flags */
#define LK_F_REPORT_WORKING 0x1u  /* worker posts WORKING (Table 1) when it picks an item up */
#define LK_F_NO_ACQUIRE     0x2u  /* skip the system-scope acquire after pickup: only for
                                     callers that never rewrite input buffers behind the
                                     GPU's caches between items (measurement variant) */
#define LK_F_ANY_PLACEMENT  0x4u  /* do not require distinct CUs for the workers */
#define LK_F_NO_LOOKAHEAD   0x8u  /* queue_depth > 1: do not read the next ring slot while an
                                     item runs (by default a worker does, and takes a command
                                     the host has already posted without another round trip) */

typedef struct lk_config {
  int32_t device;              /* HIP device ordinal */
  uint32_t n_workers;          /* 1..LK_MAX_WORKERS, at most the CU count times
                                  workers_per_cu; 0 = workers_per_cu on every CU */
  uint32_t threads_per_worker; /* 64..1024, multiple of 64; 0 = 256 (4 wave64 per CU).
                                  The workers' CUs stay shared with other kernels only as
                                  far as registers allow: a worker wave holds 104 VGPRs,
                                  so with 1024 threads (4 waves per SIMD, 416 of 512)
                                  a kernel needing more than 96 VGPRs per lane cannot
                                  run on those CUs while the context lives */
  uint32_t queue_depth;        /* 1..LK_MAX_DEPTH ring slots per mailbox; 0 = 1 */
  uint32_t cluster_policy;     /* LK_CLUSTERS_* */
  uint32_t n_clusters;         /* LK_CLUSTERS_EXPLICIT only */
  const uint32_t *cluster_of_worker; /* LK_CLUSTERS_EXPLICIT only: n_workers entries */
  uint32_t poll_sleep;         /* pause between polls, in s_sleep(1) units (64 clocks
                                  each), 0..127 */
  uint32_t flags;              /* LK_F_* */
  uint32_t log_capacity;       /* device log entries per worker (ring); 0 = no log */
  uint32_t idle_timeout_ms;    /* watchdog: a worker idle this long leaves the loop;
                                  0 = 10000 ms; at most 3600000 */
  uint32_t workers_per_cu;     /* persistent workgroups resident on one CU, 1..4 (0 = 1),
                                  each with its own mailbox; they share the CU's LDS
                                  evenly (sized so that one more never fits) and
                                  threads_per_worker x workers_per_cu must be <= 1024 so
                                  that the register file holds all of them */
  int64_t init_timeout_ns;     /* lk_init: deadline for every worker to report INIT;
                                  0 = 5 s */
  int32_t first_poll_delay;    /* pause, in s_sleep(1) units, between a worker's status
                                  record and its first read of the next command slot:
                                  LK_POLL_DELAY_ADAPTIVE (the default) learns it per worker,
                                  0 = none, 1..127 = fixed.  A read issued right after the
                                  status record usually reaches host memory before the host
                                  has posted the next command and then costs a whole PCIe
                                  round trip; the pause never delays a command that arrives
                                  later than it */
  uint32_t xcd_mask;           /* bit j set: workers only on XCD j (XCC_ID j), so the other
                                  XCDs stay free for other work (Sec. 1: work allocated on a
                                  subset of the cores); 0 = every XCD.  A context with a mask
                                  dispatches one workgroup per CU of the whole GPU, those on
                                  other XCDs leave at boot, so it needs every CU free when it
                                  starts and counts as holding all of them until disposed.
                                  n_workers = 0 then means workers_per_cu on every CU of
                                  the named XCDs; a bit beyond the device's XCDs is
                                  LK_EINVAL */
} lk_config;

#define LK_POLL_DELAY_ADAPTIVE (-1)

typedef struct lk_ctx lk_ctx;  /* opaque, owned by the library */

/* Fill *cfg with the defaults (one worker on every CU, 256 threads, depth 1, one cluster
 * per worker). */
LK_API void lk_config_default(lk_config *cfg);

/* Init phase (Sec. 3; pinning at boot, Sec. 2.3).  Checks the device, allocates the
 * mailboxes in fine-grained host-coherent memory, dispatches the persistent kernel with
 * workers_per_cu workgroups per CU on its own HSA queue and waits until every worker has
 * reported INIT (Table 1) with its physical placement.  On success *out holds a running
 * context.  Errors: LK_EINVAL (bad config, including an xcd_mask bit beyond the device's
 * XCDs or more workers than the named XCDs' CUs hold), LK_ENODEV (no device, too few free
 * CUs, workers not all resident within init_timeout_ns, more than workers_per_cu of them
 * on one CU, or a worker outside xcd_mask), LK_EHIP. */
LK_API int lk_init(const lk_config *cfg, lk_ctx **out);

/* Trigger phase (Sec. 3): post one work item to every member of `cluster`.
 * `in` and `out` are device pointers (4-byte aligned; see the op table for which are
 * used).  Both must stay valid and untouched until lk_wait returns LK_OK for the ticket.
 * `out == in` is allowed; any other overlap, or overlap with an item in flight on another
 * cluster, gives undefined results.  Non-blocking: returns LK_EAGAIN without posting
 * anything if a member's ring is full.  *ticket receives the cluster's sequence number
 * of the item (1, 2, 3, ...).  One thread at a time may submit to a given cluster.
 * Errors: LK_EINVAL (including descriptor flags the item cannot take: LK_DF_PIN_INPUT),
 * LK_EAGAIN, LK_ESTATE (disposed, or a member's worker has exited). */
LK_API int lk_submit(lk_ctx *ctx, uint32_t cluster, const lk_desc *desc, const void *in, void *out,
              uint64_t *ticket);

/* Wait phase (Sec. 3): wait until every member has reported FINISHED (Table 1) for
 * `ticket`, then release that ticket's ring slots (and those of earlier tickets of the
 * cluster).  When FINISHED is observed, the item's outputs are visible to the host and
 * to any stream.  *result (may be NULL) receives the exact int64 sum of the members'
 * partial results.  timeout_ns < 0 waits without a deadline.
 * Errors: LK_ETIMEDOUT (ticket stays valid), LK_EINVAL (ticket never posted or already
 * released), LK_EFAULT (a member rejected its descriptor), LK_ESTATE. */
LK_API int lk_wait(lk_ctx *ctx, uint32_t cluster, uint64_t ticket, int64_t timeout_ns,
            int64_t *result);

/* ------------------------------------------------------------------ batches
 * A batch is a table of tiles in device memory; every member of the cluster receives the
 * same BATCH command and the members claim tiles one at a time from a shared counter
 * (one device atomic per tile), so uneven items spread over the whole cluster inside a
 * single persistent dispatch.  Tile t runs op `op` over n elements of in/out (the same
 * bodies and layouts as the single-item ops; NOP, AFFINE_SUM_I32, SUM_I32_I64,
 * SAXPY_F32, COPY_F32 or SPIN) and writes its int64 result to partials[t].
 * lk_batch_plan cuts items into such tiles (for AXPY_F32 items, in_addr/out_addr are x and
 * the result, and the item's aux field is y). */
typedef struct lk_tile {
  uint64_t in, out;   /* device addresses of the tile's first element (4-byte aligned) */
  uint64_t in2;       /* AXPY_F32: y of the tile; 0 otherwise */
  uint32_t n;         /* elements in the tile */
  uint32_t op;        /* LK_OP_* of the tile (not BATCH) */
  int32_t a;          /* AFFINE_SUM_I32 a; SPIN iterations */
  uint32_t b;         /* AFFINE_SUM_I32 b, or the bits of SAXPY_F32 / AXPY_F32 alpha */
  uint64_t reserved;
} lk_tile; /* 48 bytes */

/* Trigger phase for a batch: `tiles` is a 16-byte aligned device array of n_tiles lk_tile
 * records and
 * `partials` a device or host-coherent int64 array of n_tiles entries; both must stay
 * untouched until lk_wait returns for the ticket.  lk_wait's result is the number of
 * tiles executed (n_tiles), summed over the members.  Errors as lk_submit. */
LK_API int lk_submit_batch(lk_ctx *ctx, uint32_t cluster, const lk_tile *tiles, uint32_t n_tiles,
                    int64_t *partials, uint64_t *ticket);

/* Cut items into tiles of at most tile_elems elements (a multiple of 256; the last tile
 * of an item may be shorter).  items: count descriptors with their in/out device
 * addresses (in_addr[i], out_addr[i]); writes up to cap tiles and, per tile, the index of
 * its item (tile_item, may be NULL); *n_tiles receives the number needed (LK_EINVAL if it
 * exceeds cap, with nothing written beyond cap). */
LK_API int lk_batch_plan(const lk_desc *items, const uint64_t *in_addr, const uint64_t *out_addr, uint32_t count,
                  uint64_t tile_elems, lk_tile *tiles, uint32_t *tile_item, uint32_t cap, uint32_t *n_tiles);

/* Timing of one completed ticket, in device wall-clock ticks (lk_info.wall_clock_hz):
 * earliest pickup and latest completion over the cluster's members. */
typedef struct lk_completion {
  int64_t result;
  uint64_t t_pick_min, t_pick_max;
  uint64_t t_done_min, t_done_max;
} lk_completion;

/* lk_wait plus the ticket's device-side timing. */
LK_API int lk_wait_info(lk_ctx *ctx, uint32_t cluster, uint64_t ticket, int64_t timeout_ns,
                 lk_completion *out);

/* Non-blocking completion test: *done = 1 if every member finished `ticket`. */
LK_API int lk_poll(lk_ctx *ctx, uint32_t cluster, uint64_t ticket, int *done);

/* Non-blocking Wait: if every member has finished `ticket`, releases it exactly as
 * lk_wait_info does (out may be NULL) and returns LK_OK; otherwise changes nothing and
 * returns LK_EAGAIN.  One call per check, for host loops that serve many clusters.
 * Errors as lk_wait_info (LK_ESTATE when a member's worker exited before finishing). */
LK_API int lk_try_wait(lk_ctx *ctx, uint32_t cluster, uint64_t ticket, lk_completion *out);

/* Hint for a host thread that drives many clusters: start fetching the cache lines it will
 * touch next for `cluster` -- the status records of `ticket` (if it is posted and not yet
 * released; 0 = none) and the command slots of the cluster's next ticket -- so that the
 * misses on lines the GPU has just written or read overlap with work on other clusters.
 * No effect on results.  Errors: LK_EINVAL, LK_ESTATE. */
LK_API int lk_prefetch(lk_ctx *ctx, uint32_t cluster, uint64_t ticket);

/* Dispose phase (Sec. 3; THREAD_EXIT, Table 1): post EXIT to every worker, wait for the
 * persistent kernel to end, copy the device log to the host and free every GPU
 * resource.  Idempotent.  The context object itself stays readable (lk_info,
 * lk_topology, lk_read_log) until lk_free.  Errors: LK_ETIMEDOUT if the kernel did not
 * end in time (the context is then poisoned and its GPU resources are leaked). */
LK_API int lk_dispose(lk_ctx *ctx);

/* Release the context object (after lk_dispose; calls it first if needed). */
LK_API int lk_free(lk_ctx *ctx);

/* ------------------------------------------------------------------ introspection */
typedef struct lk_info {
  uint32_t n_workers, n_clusters, queue_depth, threads_per_worker;
  uint32_t cu_count, xcd_count;
  uint32_t state;              /* 0 running, 1 disposed, 2 poisoned */
  uint32_t workers_exited;     /* workers that left the loop (EXIT or watchdog) */
  uint64_t wall_clock_hz;      /* device wall-clock rate */
  double init_ms;              /* lk_init duration */
  double dispose_ms;           /* lk_dispose duration (0 before) */
  double kernel_ms;            /* persistent kernel duration from the packet processor's
                                  dispatch timestamps (after lk_dispose; 0 before, and 0
                                  when a tool intercepting the queue hides them) */
  double device_span_ms;       /* first worker boot to last worker exit on the device
                                  wall clock (after lk_dispose) */
  uint32_t workers_per_cu;     /* as configured */
  uint32_t max_workers_on_a_cu; /* most workers found on one physical CU at boot */
  uint32_t pin_capacity;       /* bytes of x one worker can keep pinned (LK_DF_PIN_INPUT) */
  uint32_t xcd_mask;           /* XCDs holding workers (every XCD unless the config named some) */
} lk_info;

LK_API int lk_get_info(lk_ctx *ctx, lk_info *info);

/* Physical placement of worker w, read from the HW_ID / XCC_ID registers at boot: the
 * check Sec. 2.3 makes, that each persistent block sits on the core it was meant for
 * (there, that the hardware placed the blocks round-robin, one per SM; here the
 * workgroups' own hardware ids, from which the host orders the workers).  The worker's
 * XCD, shader engine, shader array and CU index go to the non-NULL outputs.
 * Errors: LK_EINVAL (NULL context or worker out of range). */
LK_API int lk_topology(lk_ctx *ctx, uint32_t worker, uint32_t *xcc, uint32_t *se, uint32_t *sh,
                uint32_t *cu);

/* Members of a cluster, in slice order.  *count receives the member count; up to `cap`
 * worker indices are written to `workers`. */
LK_API int lk_cluster_members(lk_ctx *ctx, uint32_t cluster, uint32_t *workers, uint32_t cap,
                       uint32_t *count);

/* Device log, one record per executed command (available after lk_dispose). */
typedef struct lk_log_entry {
  uint32_t seq;       /* mailbox sequence number = the cluster's ticket */
  uint16_t code;      /* command code: 4 NOP, 8 EXIT, 16 + op WORK (Table 1) */
  uint16_t worker;    /* worker index */
  uint32_t xcc;       /* XCC_ID read when the command was picked up */
  uint32_t hwid;      /* HW_ID read when the command was picked up */
  uint64_t t_pick;    /* device wall clock at pickup */
  uint64_t t_done;    /* device wall clock before the completion was published */
} lk_log_entry;

/* Copy up to `cap` of worker w's most recent log records (oldest first) into `out`;
 * *count receives the number written.  Valid after lk_dispose. */
LK_API int lk_read_log(lk_ctx *ctx, uint32_t worker, lk_log_entry *out, uint32_t cap,
                uint32_t *count);

/* Item slicing rule (see "clusters" above) as a pure host function. */
LK_API int lk_slice(uint64_t n, uint32_t k, uint32_t j, uint64_t *lo, uint64_t *hi);

LK_API const char *lk_strerror(int code);
/* Detail of the calling thread's most recent failure ("" if none). */
LK_API const char *lk_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* LK_H */
