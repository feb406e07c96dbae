/*
 * lk_host.cpp -- host side of the LightKernel dispatch library (include/lk.h).
 *
 * Phases (Sec. 3): lk_init boots the persistent kernel (Init), lk_submit posts a command
 * into each member's to_GPU mailbox (Trigger), lk_wait polls the members' from_GPU
 * mailboxes (Wait), lk_dispose posts THREAD_EXIT and joins the kernel (Dispose).
 *
 * Submit and wait make no HIP runtime call and no driver transfer: the mailboxes live in
 * fine-grained host-coherent memory that the workers read and write directly over PCIe,
 * so the host side of a dispatch is a handful of ordinary stores and loads.
 */
#include <immintrin.h>

#include <algorithm>
#include <chrono>
#include <cstdarg>
#include <map>
#include <mutex>
#include <cstdio>
#include <cstring>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "lk.h"
#include "lk_backend.h"
#include "lk_common.h"
#include "lk_error.h"
#include "lk_wire.h"

namespace {

thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

}  // namespace

void lkh::set_last_error(const char *msg) { g_last_error = msg ? msg : ""; }

namespace {

using clk = std::chrono::steady_clock;

inline uint64_t load_acquire(const uint64_t *p) { return __atomic_load_n(p, __ATOMIC_ACQUIRE); }
inline void store_relaxed(uint64_t *p, uint64_t v) { __atomic_store_n(p, v, __ATOMIC_RELAXED); }
inline void store_release(uint64_t *p, uint64_t v) { __atomic_store_n(p, v, __ATOMIC_RELEASE); }

enum State : uint32_t { RUNNING = 0, DISPOSED = 1, POISONED = 2 };

struct WorkerInfo {
  uint32_t mailbox;
  uint32_t hwid, xcc, se, sh, cu;
};

// Host-side sequence state of one cluster, on its own 128-byte block: clusters are
// driven by different host threads and must not share cache lines.
struct alignas(128) ClusterSeq {
  uint64_t posted = 0;    // last ticket posted (== every member mailbox's last seq)
  uint64_t consumed = 0;  // last ticket whose completion the host has taken
};

// A decoded status record.
struct Status {
  uint32_t code;
  int64_t partial;
  uint64_t t_pick, t_done;
};

inline bool exited_code(uint32_t code) { return code == LKW_FROM_EXITED || code == LKW_FROM_TIMEDOUT; }

// Workers of the live persistent dispatches of this process, per device.  Every worker
// holds a whole CU until its dispatch ends, so a context that would need more CUs than
// are left can never boot: lk_init refuses it at once instead of timing out.
std::mutex g_cu_mutex;
std::map<int, uint32_t> g_cu_in_use;

bool reserve_cus(int device, uint32_t n, uint32_t cu_count, uint32_t *in_use) {
  std::lock_guard<std::mutex> lock(g_cu_mutex);
  uint32_t &u = g_cu_in_use[device];
  *in_use = u;
  if (u + n > cu_count) return false;
  u += n;
  return true;
}

void release_cus(int device, uint32_t n) {
  std::lock_guard<std::mutex> lock(g_cu_mutex);
  uint32_t &u = g_cu_in_use[device];
  u = u >= n ? u - n : 0;
}

}  // namespace

struct lk_ctx {
  lk_config cfg{};
  int device = 0;
  uint32_t n_workers = 0, depth = 1, threads = 256, n_clusters = 0, cu_count = 0, xcd_count = 0;
  // Ring arithmetic of every submit and wait, without a division on the common path:
  // slots per mailbox, and depth - 1 when the depth is a power of two (else 0).
  uint64_t stride = 1;
  uint32_t depth_mask = 0;
  bool depth_pow2 = true;
  uint32_t per_cu = 1, max_on_a_cu = 0;
  uint32_t cus_held = 0;  // CUs counted for this context in the process registry
  uint32_t pin_bytes = 0; // dynamic LDS of each worker: the largest x slice it can pin
  uint32_t xcd_mask = 0;  // XCDs that hold workers (every XCD when the config names none)
  bool masked = false;    // xcd_mask leaves some XCD out: the dispatch spans every CU
  uint32_t log_cap = 0;
  uint64_t wall_hz = 100000000ull;
  State state = RUNNING;
  lkbe::Dispatch *wq = nullptr;  // the persistent dispatch (its own hardware queue)
  void *host_region = nullptr;
  lkw_cmd *cmd = nullptr;
  lkw_status *status = nullptr;
  lkw_worker *wrec = nullptr;
  lkw_log *d_log = nullptr;
  uint32_t *d_claim = nullptr;
  uint64_t *d_batch_counters = nullptr;             // [cluster][depth], 128 bytes apart
  std::vector<uint64_t> batch_base;                 // [cluster][depth], host copy of each base
  std::vector<WorkerInfo> workers;                  // physical order
  std::vector<std::vector<uint32_t>> clusters;      // member worker indices, slice order
  std::vector<std::vector<uint32_t>> cluster_mbox;  // member mailboxes, slice order
  std::vector<ClusterSeq> seqs;                     // per cluster
  std::vector<uint32_t> cluster_of_mbox;
  std::vector<lkw_log> host_log;                    // copied at dispose
  double init_ms = 0, dispose_ms = 0, kernel_ms = 0, device_span_ms = 0;
  bool cus_reserved = false;  // counted in g_cu_in_use until the dispatch has ended
  bool kernel_launched = false;
  uint32_t exited_at_dispose = 0;
};

namespace {

inline uint64_t ring_slot(const lk_ctx *c, uint64_t seq) {
  return c->depth_pow2 ? (seq & c->depth_mask) : seq % c->depth;
}
lkw_cmd *slot_cmd(lk_ctx *c, uint32_t mb, uint64_t seq) {
  return c->cmd + static_cast<uint64_t>(mb) * c->stride + ring_slot(c, seq);
}
lkw_status *slot_status(lk_ctx *c, uint32_t mb, uint64_t seq) {
  return c->status + static_cast<uint64_t>(mb) * c->stride + ring_slot(c, seq);
}

// True (and *out filled) once the status record of `seq` is complete: word 0 holds seq
// with a final code and every other word carries seq's tag.
bool read_status(const lkw_status *st, uint64_t seq, Status *out) {
  const uint64_t w0 = load_acquire(&st->w[LKW_S_WORD]);
  if (LKW_SEQ(w0) != seq || LKW_CODE(w0) == LKW_FROM_WORKING) return false;
  uint64_t v[LKW_S_WORDS];
  const uint64_t tag = LKW_TAG(seq);
  for (int i = 1; i < LKW_S_WORDS; ++i) {
    v[i] = __atomic_load_n(&st->w[i], __ATOMIC_ACQUIRE);
    if ((v[i] & ~LKW_PAYLOAD_MASK) != tag) return false;
  }
  if (out) {
    out->code = LKW_CODE(w0);
    out->partial = static_cast<int64_t>((v[LKW_S_PART_LO] & 0xffffffffull) | ((v[LKW_S_PART_HI] & 0xffffffffull) << 32));
    out->t_pick = v[LKW_S_T_PICK] & LKW_PAYLOAD_MASK;
    out->t_done = v[LKW_S_T_DONE] & LKW_PAYLOAD_MASK;
  }
  return true;
}
uint32_t worker_code(lk_ctx *c, uint32_t mb) { return LKW_CODE(load_acquire(&c->wrec[mb].word)); }

// Write one command slot: tagged payload words first, then the doorbell word (release).
void post_cmd(lk_ctx *c, uint32_t mb, uint64_t seq, uint32_t code, uint64_t n, uint64_t in, uint64_t out,
              uint64_t aux, uint32_t a, uint32_t b, float alpha, uint32_t member, uint32_t dflags = 0) {
  lkw_cmd *s = slot_cmd(c, mb, seq);
  const uint64_t tag = LKW_TAG(seq);
  uint32_t alpha_bits;
  memcpy(&alpha_bits, &alpha, 4);
  store_relaxed(&s->w[LKW_W_N], tag | (n & LKW_PAYLOAD_MASK));
  store_relaxed(&s->w[LKW_W_IN], tag | (in & LKW_PAYLOAD_MASK));
  store_relaxed(&s->w[LKW_W_OUT], tag | (out & LKW_PAYLOAD_MASK));
  store_relaxed(&s->w[LKW_W_AUX], tag | (aux & LKW_PAYLOAD_MASK));
  store_relaxed(&s->w[LKW_W_A], tag | (static_cast<uint64_t>(member & 0xffffu) << 32) | a);
  store_relaxed(&s->w[LKW_W_B], tag | (static_cast<uint64_t>(dflags & 0xffffu) << 32) | b);
  store_relaxed(&s->w[LKW_W_ALPHA], tag | alpha_bits);
  store_release(&s->w[LKW_W_DOORBELL], LKW_WORD(seq, code));
}

bool op_reads(uint32_t op) {
  return op == LK_OP_AFFINE_SUM_I32 || op == LK_OP_SUM_I32_I64 || op == LK_OP_SAXPY_F32 || op == LK_OP_COPY_F32 ||
         op == LK_OP_AXPY_F32;
}
bool op_writes(uint32_t op) {
  return op == LK_OP_AFFINE_SUM_I32 || op == LK_OP_SAXPY_F32 || op == LK_OP_COPY_F32 || op == LK_OP_AXPY_F32;
}
bool op_has_result(uint32_t op) { return op == LK_OP_AFFINE_SUM_I32 || op == LK_OP_SUM_I32_I64; }

int validate_config(const lk_config *cfg) {
  if (!cfg) return fail(LK_EINVAL, "config is NULL");
  if (cfg->n_workers > LK_MAX_WORKERS) return fail(LK_EINVAL, "n_workers %u > %u", cfg->n_workers, LK_MAX_WORKERS);
  const uint32_t t = cfg->threads_per_worker;
  if (t != 0 && (t < 64 || t > 1024 || t % 64 != 0))
    return fail(LK_EINVAL, "threads_per_worker %u: need a multiple of 64 in 64..1024", t);
  const uint32_t wpc = cfg->workers_per_cu ? cfg->workers_per_cu : 1;
  if (wpc > LK_MAX_WORKERS_PER_CU) return fail(LK_EINVAL, "workers_per_cu %u > %u", wpc, LK_MAX_WORKERS_PER_CU);
  if (wpc * (t ? t : 256) > 1024)
    return fail(LK_EINVAL, "threads_per_worker %u x workers_per_cu %u > 1024: not every worker could stay resident",
                t ? t : 256, wpc);
  if (cfg->queue_depth > LK_MAX_DEPTH) return fail(LK_EINVAL, "queue_depth %u > %u", cfg->queue_depth, LK_MAX_DEPTH);
  if (cfg->cluster_policy > LK_CLUSTERS_EXPLICIT) return fail(LK_EINVAL, "unknown cluster_policy %u", cfg->cluster_policy);
  if (cfg->cluster_policy == LK_CLUSTERS_EXPLICIT) {
    if (!cfg->cluster_of_worker || cfg->n_clusters == 0)
      return fail(LK_EINVAL, "explicit clusters need cluster_of_worker and n_clusters > 0");
    if (cfg->n_workers == 0) return fail(LK_EINVAL, "explicit clusters need an explicit n_workers");
    std::vector<uint32_t> seen(cfg->n_clusters, 0);
    for (uint32_t w = 0; w < cfg->n_workers; ++w) {
      if (cfg->cluster_of_worker[w] >= cfg->n_clusters)
        return fail(LK_EINVAL, "cluster_of_worker[%u] = %u out of range", w, cfg->cluster_of_worker[w]);
      seen[cfg->cluster_of_worker[w]] = 1;
    }
    for (uint32_t k = 0; k < cfg->n_clusters; ++k)
      if (!seen[k]) return fail(LK_EINVAL, "cluster %u has no worker", k);
  }
  if (cfg->poll_sleep > 127) return fail(LK_EINVAL, "poll_sleep %u > 127", cfg->poll_sleep);
  if (cfg->idle_timeout_ms > 3600000u) return fail(LK_EINVAL, "idle_timeout_ms %u > 3600000", cfg->idle_timeout_ms);
  if (cfg->flags & ~(LK_F_REPORT_WORKING | LK_F_NO_ACQUIRE | LK_F_ANY_PLACEMENT | LK_F_NO_LOOKAHEAD))
    return fail(LK_EINVAL, "unknown flags 0x%x", cfg->flags);
  if (cfg->init_timeout_ns < 0) return fail(LK_EINVAL, "init_timeout_ns < 0");
  if (cfg->log_capacity > (1u << 24)) return fail(LK_EINVAL, "log_capacity %u > 2^24", cfg->log_capacity);
  if (cfg->first_poll_delay < LK_POLL_DELAY_ADAPTIVE || cfg->first_poll_delay > 127)
    return fail(LK_EINVAL, "first_poll_delay %d: need -1 (adaptive) or 0..127", cfg->first_poll_delay);
  return LK_OK;
}

// Only called once the persistent dispatch has ended (or was never made).
void release_gpu(lk_ctx *c) {
  if (c->cus_reserved) release_cus(c->device, c->cus_held);
  c->cus_reserved = false;
  delete c->wq;
  c->wq = nullptr;
  lkbe::device_free(c->d_batch_counters);
  c->d_batch_counters = nullptr;
  lkbe::device_free(c->d_log);
  lkbe::device_free(c->d_claim);
  lkbe::host_free(c->host_region);
  c->d_log = nullptr;
  c->d_claim = nullptr;
  c->host_region = nullptr;
  c->cmd = nullptr;
  c->status = nullptr;
  c->wrec = nullptr;
}

// Wait (bounded) for the persistent kernel to end; true if it did.
bool join_kernel(lk_ctx *c, double seconds) {
  const auto deadline = clk::now() + std::chrono::duration<double>(seconds);
  for (;;) {
    if (!c->wq || c->wq->finished()) return true;
    if (clk::now() > deadline) return false;
    std::this_thread::sleep_for(std::chrono::microseconds(200));
  }
}

}  // namespace

extern "C" {

void lk_config_default(lk_config *cfg) {
  if (!cfg) return;
  memset(cfg, 0, sizeof *cfg);
  cfg->threads_per_worker = 256;
  cfg->queue_depth = 1;
  cfg->cluster_policy = LK_CLUSTERS_PER_WORKER;
  cfg->log_capacity = 0;
  cfg->idle_timeout_ms = 10000;
  cfg->workers_per_cu = 1;
  cfg->first_poll_delay = LK_POLL_DELAY_ADAPTIVE;
}

int lk_slice(uint64_t n, uint32_t k, uint32_t j, uint64_t *lo, uint64_t *hi) {
  if (!lo || !hi) return fail(LK_EINVAL, "lo/hi is NULL");
  if (k == 0) return fail(LK_EINVAL, "k == 0");
  lkd::slice_bounds(n, k, j, lo, hi);
  return LK_OK;
}

const char *lk_strerror(int code) {
  switch (code) {
    case LK_OK: return "ok";
    case LK_EINVAL: return "invalid argument";
    case LK_EAGAIN: return "mailbox ring full";
    case LK_ETIMEDOUT: return "timed out";
    case LK_ESTATE: return "invalid state";
    case LK_ENODEV: return "no usable device";
    case LK_EHIP: return "HIP runtime error";
    case LK_EFAULT: return "descriptor rejected by worker";
    default: return "unknown error";
  }
}

const char *lk_last_error(void) { return g_last_error.c_str(); }

int lk_init(const lk_config *cfg_in, lk_ctx **out) {
  const auto t_begin = clk::now();
  if (!out) return fail(LK_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = validate_config(cfg_in);
  if (rc) return rc;
  lk_config cfg = *cfg_in;

  lkbe::DeviceInfo dev;
  {
    std::string err;
    if ((rc = lkbe::device_info(cfg.device, &dev, &err)) != LK_OK) return fail(rc, "%s", err.c_str());
  }

  auto *c = new lk_ctx();
  c->cfg = cfg;
  c->cfg.cluster_of_worker = nullptr;
  c->device = cfg.device;
  c->cu_count = dev.cu_count;
  c->per_cu = cfg.workers_per_cu ? cfg.workers_per_cu : 1;
  // XCD restriction: workers only on the named XCDs (equal CU counts per XCD).
  const uint32_t nx = dev.xcc_count ? dev.xcc_count : 1;
  const uint32_t all_xcd = nx >= 32 ? ~0u : (1u << nx) - 1u;
  if (cfg.xcd_mask & ~all_xcd) {
    delete c;
    return fail(LK_EINVAL, "xcd_mask 0x%x names an XCD beyond the device's %u", cfg.xcd_mask, nx);
  }
  c->xcd_mask = cfg.xcd_mask ? cfg.xcd_mask : all_xcd;
  c->masked = c->xcd_mask != all_xcd;
  const uint32_t cus_usable =
      c->masked ? c->cu_count / nx * static_cast<uint32_t>(__builtin_popcount(c->xcd_mask)) : c->cu_count;
  c->n_workers = cfg.n_workers ? cfg.n_workers : cus_usable * c->per_cu;
  c->depth = cfg.queue_depth ? cfg.queue_depth : 1;
  c->stride = LKW_RING_STRIDE(c->depth);
  c->depth_pow2 = (c->depth & (c->depth - 1)) == 0;
  c->depth_mask = c->depth_pow2 ? c->depth - 1 : 0;
  c->threads = cfg.threads_per_worker ? cfg.threads_per_worker : 256;
  c->log_cap = cfg.log_capacity;
  if (c->n_workers > cus_usable * c->per_cu || c->n_workers > LK_MAX_WORKERS) {
    const uint32_t cap = std::min(cus_usable * c->per_cu, LK_MAX_WORKERS);
    const bool masked = c->masked;
    delete c;
    return fail(LK_EINVAL, "n_workers %u exceeds %u (%u per CU%s)", cfg.n_workers, cap,
                cfg.workers_per_cu ? cfg.workers_per_cu : 1, masked ? " of the masked XCDs" : "");
  }
  // Dynamic LDS per worker: one worker per CU takes 96 KiB, so a second never fits;
  // k workers per CU take an even share of the CU's LDS less 2 KiB (room for the static
  // LDS and the allocation granule), so k fit and k + 1 do not.
  const uint32_t lds_cu = dev.lds_per_cu;
  const uint32_t lds_pad = c->per_cu == 1 ? LKW_LDS_PAD_BYTES : (lds_cu / c->per_cu - 2048u) / 256u * 256u;
  c->pin_bytes = lds_pad;
  {
    // Until the hardware ids are known every worker may sit on a CU of its own; a masked
    // context dispatches over every CU.
    uint32_t in_use = 0;
    c->cus_held = c->masked ? c->cu_count : std::min(c->n_workers, c->cu_count);
    if (!reserve_cus(cfg.device, c->cus_held, c->cu_count, &in_use)) {
      const uint32_t want = c->cus_held, cus = c->cu_count;
      delete c;
      return fail(LK_ENODEV, "%u CUs needed but this process's running contexts already hold %u of the %u CUs", want,
                  in_use, cus);
    }
    c->cus_reserved = true;
  }
  c->wall_hz = dev.wall_hz;

  auto bail = [&](int code) {
    release_gpu(c);
    delete c;
    return code;
  };

  // Mailboxes: command ring, status ring, worker records, in one host-coherent region.
  const size_t cmd_bytes = sizeof(lkw_cmd) * c->n_workers * LKW_RING_STRIDE(c->depth);
  const size_t st_bytes = sizeof(lkw_status) * c->n_workers * LKW_RING_STRIDE(c->depth);
  const size_t wr_bytes = sizeof(lkw_worker) * c->n_workers;
  auto up = [](size_t v) { return (v + 4095) & ~static_cast<size_t>(4095); };
  const size_t region = up(cmd_bytes) + up(st_bytes) + up(wr_bytes);
  std::string err;
  if ((rc = lkbe::host_alloc(cfg.device, region, &c->host_region, &err)) != LK_OK)
    return bail(fail(rc, "mailboxes: %s", err.c_str()));
  char *base = static_cast<char *>(c->host_region);
  c->cmd = reinterpret_cast<lkw_cmd *>(base);
  c->status = reinterpret_cast<lkw_status *>(base + up(cmd_bytes));
  c->wrec = reinterpret_cast<lkw_worker *>(base + up(cmd_bytes) + up(st_bytes));
  // Mark every worker record as not yet booted (INIT is 0, so use an impossible word).
  for (uint32_t m = 0; m < c->n_workers; ++m) store_release(&c->wrec[m].word, LKW_WORD(~0ull >> 8, 0xffu));

  if ((rc = lkbe::device_alloc(cfg.device, 256, reinterpret_cast<void **>(&c->d_claim), &err)) != LK_OK)
    return bail(fail(rc, "claim counter: %s", err.c_str()));
  // Tile counters of batches: one per (cluster, ring slot) -- there are at most n_workers
  // clusters -- 128 bytes apart and never reset: each batch advances its counter by
  // n_tiles + members (every member's last claim overshoots once), which the host adds to
  // that slot's base.
  {
    const size_t cb = static_cast<size_t>(c->n_workers) * c->depth * 128;
    if ((rc = lkbe::device_alloc(cfg.device, cb, reinterpret_cast<void **>(&c->d_batch_counters), &err)) != LK_OK)
      return bail(fail(rc, "batch counters: %s", err.c_str()));
  }
  if (c->log_cap) {
    const size_t lb = sizeof(lkw_log) * c->n_workers * static_cast<size_t>(c->log_cap);
    if ((rc = lkbe::device_alloc(cfg.device, lb, reinterpret_cast<void **>(&c->d_log), &err)) != LK_OK)
      return bail(fail(rc, "log: %s", err.c_str()));
  }

  // The persistent worker runs on a hardware queue of its own.
  if (!(c->wq = lkbe::open_dispatch(cfg.device, &err))) return bail(fail(LK_EHIP, "worker queue: %s", err.c_str()));

  lkw_params p{};
  p.cmd = c->cmd;
  p.status = c->status;
  p.workers = c->wrec;
  p.log = c->d_log;
  p.claim = c->d_claim;
  p.n_workers = c->n_workers;
  p.depth = c->depth;
  p.log_cap = c->log_cap ? c->log_cap : 1;
  p.poll_sleep = cfg.poll_sleep;
  p.threads = c->threads;
  p.flags = ((cfg.flags & LK_F_REPORT_WORKING) ? LKW_K_REPORT_WORKING : 0u) |
            ((cfg.flags & LK_F_NO_ACQUIRE) ? LKW_K_NO_ACQUIRE : 0u) |
            ((cfg.flags & LK_F_NO_LOOKAHEAD) ? LKW_K_NO_LOOKAHEAD : 0u);
  const uint32_t idle_ms = cfg.idle_timeout_ms ? cfg.idle_timeout_ms : 10000u;
  p.idle_ticks = c->wall_hz / 1000ull * idle_ms;
  p.first_delay = cfg.first_poll_delay;
  p.b2b_ticks = static_cast<uint32_t>(c->wall_hz / 100000ull);  // 10 us
  p.lds_bytes = lds_pad;
  // About a host round trip (1.6 us): a look-ahead read waits at most that long, so it
  // is issued only when the previous item ran longer and the read hides under the item.
  p.la_ticks = static_cast<uint32_t>(c->wall_hz / 625000ull);
  p.xcc_mask = c->masked ? c->xcd_mask : ~0u;

  // A masked context dispatches one workgroup per CU slot of the whole GPU; the ones on
  // other XCDs leave at once (and so do any beyond n_workers).
  const uint32_t grid = c->masked ? c->cu_count * c->per_cu : c->n_workers;
  if (!c->wq->start(p, grid, c->threads, lds_pad, &err))
    return bail(fail(LK_EHIP, "persistent worker dispatch: %s", err.c_str()));
  c->kernel_launched = true;

  // Boot handshake: every worker reports INIT with its placement.
  const int64_t to_ns = cfg.init_timeout_ns ? cfg.init_timeout_ns : 5000000000ll;
  const auto deadline = clk::now() + std::chrono::nanoseconds(to_ns);
  uint32_t booted = 0;
  bool early_end = false;
  while (booted < c->n_workers) {
    booted = 0;
    for (uint32_t m = 0; m < c->n_workers; ++m) booted += load_acquire(&c->wrec[m].word) == LKW_WORD(0, LKW_FROM_INIT);
    if (booted == c->n_workers) break;
    if (c->wq->finished()) {
      early_end = true;
      break;
    }
    if (clk::now() > deadline) break;
    _mm_pause();
  }
  if (booted < c->n_workers) {
    for (uint32_t m = 0; m < c->n_workers; ++m) post_cmd(c, m, 1, LKW_TO_EXIT, 0, 0, 0, 0, 0, 0, 0.f, 0);
    const double wait_s = 2.0 + idle_ms / 1000.0;
    if (!join_kernel(c, wait_s)) {
      c->state = POISONED;
      *out = c;  // resources cannot be freed while the kernel may still touch them
      return fail(LK_ENODEV, "only %u of %u workers became resident; kernel did not end (context poisoned)",
                  booted, c->n_workers);
    }
    const int code = fail(LK_ENODEV, "only %u of %u workers became resident within %.3f s%s", booted,
                          c->n_workers, to_ns / 1e9, early_end ? " (kernel ended early)" : "");
    return bail(code);
  }

  // Placement learnt from the hardware-id registers; workers in physical order.
  std::vector<WorkerInfo> ws(c->n_workers);
  for (uint32_t m = 0; m < c->n_workers; ++m) {
    const uint32_t hw = __atomic_load_n(&c->wrec[m].hwid, __ATOMIC_ACQUIRE);
    const uint32_t xcc = __atomic_load_n(&c->wrec[m].xcc, __ATOMIC_ACQUIRE) & 0xfu;
    ws[m] = WorkerInfo{m, hw, xcc, (hw >> 13) & 3u, (hw >> 12) & 1u, (hw >> 8) & 15u};
  }
  std::sort(ws.begin(), ws.end(), [](const WorkerInfo &x, const WorkerInfo &y) {
    return std::make_tuple(x.xcc, x.se, x.sh, x.cu, x.mailbox) < std::make_tuple(y.xcc, y.se, y.sh, y.cu, y.mailbox);
  });
  // Workers per physical CU (sorted, so co-resident workers are adjacent).
  for (uint32_t i = 0, run = 0; i < c->n_workers; ++i) {
    const bool same = i > 0 && ws[i - 1].xcc == ws[i].xcc && ws[i - 1].se == ws[i].se && ws[i - 1].sh == ws[i].sh &&
                      ws[i - 1].cu == ws[i].cu;
    run = same ? run + 1 : 1;
    c->max_on_a_cu = std::max(c->max_on_a_cu, run);
  }
  for (const WorkerInfo &w : ws)
    if (!((c->xcd_mask >> w.xcc) & 1u)) {  // cannot happen unless XCC_ID disagrees with the mask's numbering
      for (uint32_t m = 0; m < c->n_workers; ++m) post_cmd(c, m, 1, LKW_TO_EXIT, 0, 0, 0, 0, 0, 0, 0.f, 0);
      if (!join_kernel(c, 2.0 + idle_ms / 1000.0)) {
        c->state = POISONED;
        *out = c;
        return fail(LK_ENODEV, "a worker booted on XCD %u outside xcd_mask 0x%x; kernel did not end", w.xcc,
                    c->xcd_mask);
      }
      return bail(fail(LK_ENODEV, "a worker booted on XCD %u outside xcd_mask 0x%x", w.xcc, c->xcd_mask));
    }
  if (!(cfg.flags & LK_F_ANY_PLACEMENT) && c->max_on_a_cu > c->per_cu) {
    for (uint32_t m = 0; m < c->n_workers; ++m) post_cmd(c, m, 1, LKW_TO_EXIT, 0, 0, 0, 0, 0, 0, 0.f, 0);
    if (!join_kernel(c, 2.0 + idle_ms / 1000.0)) {
      c->state = POISONED;
      *out = c;
      return fail(LK_ENODEV, "%u workers share one CU (at most %u asked); kernel did not end", c->max_on_a_cu,
                  c->per_cu);
    }
    return bail(fail(LK_ENODEV, "%u workers share one CU (at most %u asked)", c->max_on_a_cu, c->per_cu));
  }
  c->workers = ws;
  {
    std::vector<uint32_t> xs;
    for (auto &w : ws) xs.push_back(w.xcc);
    std::sort(xs.begin(), xs.end());
    c->xcd_count = static_cast<uint32_t>(std::unique(xs.begin(), xs.end()) - xs.begin());
  }

  // Clusters.
  switch (cfg.cluster_policy) {
    case LK_CLUSTERS_PER_WORKER:
      for (uint32_t w = 0; w < c->n_workers; ++w) c->clusters.push_back({w});
      break;
    case LK_CLUSTERS_ONE: {
      std::vector<uint32_t> all(c->n_workers);
      for (uint32_t w = 0; w < c->n_workers; ++w) all[w] = w;
      c->clusters.push_back(all);
      break;
    }
    case LK_CLUSTERS_PER_XCD: {
      uint32_t prev = ~0u;
      for (uint32_t w = 0; w < c->n_workers; ++w) {
        if (ws[w].xcc != prev) c->clusters.emplace_back();
        c->clusters.back().push_back(w);
        prev = ws[w].xcc;
      }
      break;
    }
    case LK_CLUSTERS_EXPLICIT:
      c->clusters.resize(cfg.n_clusters);
      for (uint32_t w = 0; w < c->n_workers; ++w) c->clusters[cfg.cluster_of_worker[w]].push_back(w);
      break;
  }
  c->n_clusters = static_cast<uint32_t>(c->clusters.size());
  c->cluster_mbox.resize(c->n_clusters);
  c->cluster_of_mbox.assign(c->n_workers, 0);
  for (uint32_t k = 0; k < c->n_clusters; ++k)
    for (uint32_t w : c->clusters[k]) {
      c->cluster_mbox[k].push_back(ws[w].mailbox);
      c->cluster_of_mbox[ws[w].mailbox] = k;
    }
  c->seqs.assign(c->n_clusters, ClusterSeq{});
  c->batch_base.assign(static_cast<size_t>(c->n_clusters) * c->depth, 0);
  c->init_ms = std::chrono::duration<double, std::milli>(clk::now() - t_begin).count();
  *out = c;
  g_last_error.clear();
  return LK_OK;
}

int lk_submit(lk_ctx *c, uint32_t cluster, const lk_desc *d, const void *in, void *out, uint64_t *ticket) {
  if (!c || !d || !ticket) return fail(LK_EINVAL, "NULL argument");
  if (c->state != RUNNING) return fail(LK_ESTATE, "context is not running");
  if (cluster >= c->n_clusters) return fail(LK_EINVAL, "cluster %u of %u", cluster, c->n_clusters);
  if (d->op >= LK_OP_COUNT) return fail(LK_EINVAL, "unknown op %u", d->op);
  if (d->op == LK_OP_BATCH) return fail(LK_EINVAL, "batches go through lk_submit_batch");
  if (d->reserved) return fail(LK_EINVAL, "reserved must be 0");
  if (d->flags & ~(LK_DF_PIN_INPUT | LK_DF_PIN_RELOAD)) return fail(LK_EINVAL, "unknown descriptor flags 0x%x", d->flags);
  if (d->n > LK_MAX_N) return fail(LK_EINVAL, "n %llu > LK_MAX_N", static_cast<unsigned long long>(d->n));
  const uint64_t ia = reinterpret_cast<uint64_t>(in), oa = reinterpret_cast<uint64_t>(out);
  if (d->n && op_reads(d->op) && (!in || (ia & 3u))) return fail(LK_EINVAL, "input pointer NULL or not 4-byte aligned");
  if (d->n && op_writes(d->op) && (!out || (oa & 3u))) return fail(LK_EINVAL, "output pointer NULL or not 4-byte aligned");
  if ((ia | oa | d->aux) >> LKW_TAG_SHIFT) return fail(LK_EINVAL, "pointer outside the 48-bit address range");
  if (d->op == LK_OP_AXPY_F32) {
    if (d->n && (!d->aux || (d->aux & 3u))) return fail(LK_EINVAL, "AXPY_F32 needs y (aux) 4-byte aligned");
  } else if (d->aux & 7u) {
    return fail(LK_EINVAL, "aux not 8-byte aligned");
  }
  if (d->op == LK_OP_SPIN && d->a < 0) return fail(LK_EINVAL, "SPIN iterations < 0");

  const std::vector<uint32_t> &mbs = c->cluster_mbox[cluster];
  ClusterSeq &cs = c->seqs[cluster];
  const uint64_t t = cs.posted + 1;
  if (t - cs.consumed > c->depth) return fail(LK_EAGAIN, "ring full (depth %u)", c->depth);
  for (uint32_t mb : mbs)
    if (exited_code(worker_code(c, mb))) return fail(LK_ESTATE, "worker of mailbox %u has exited", mb);

  const uint32_t k = static_cast<uint32_t>(mbs.size());
  const uint32_t esz = 4;
  if (d->flags && d->n) {
    if (d->op != LK_OP_SAXPY_F32 && d->op != LK_OP_AXPY_F32 && d->op != LK_OP_AFFINE_SUM_I32 &&
        d->op != LK_OP_SUM_I32_I64)
      return fail(LK_EINVAL, "pinned input needs SAXPY_F32, AXPY_F32, AFFINE_SUM_I32 or SUM_I32_I64, not op %u", d->op);
    const uint64_t used_out = d->op == LK_OP_SUM_I32_I64 ? 0 : oa;  // SUM reads x only
    if ((ia | used_out | (d->op == LK_OP_AXPY_F32 ? d->aux : 0)) & 15u)
      return fail(LK_EINVAL, "pinned input needs 16-byte aligned in, out and y");
    for (uint32_t j = 0; j < k; ++j) {
      uint64_t lo, hi;
      lkd::slice_bounds(d->n, k, j, &lo, &hi);
      if ((hi - lo) & 3u)
        return fail(LK_EINVAL, "pinned input: member %u slice of %llu elements is not a multiple of 4", j,
                    static_cast<unsigned long long>(hi - lo));
      if ((hi - lo) * esz > c->pin_bytes)
        return fail(LK_EINVAL, "pinned input: member %u slice of %llu bytes exceeds the %u-byte LDS buffer", j,
                    static_cast<unsigned long long>((hi - lo) * esz), c->pin_bytes);
    }
  }
  for (uint32_t j = 0; j < k; ++j) {
    uint64_t lo, hi;
    lkd::slice_bounds(d->n, k, j, &lo, &hi);
    const uint64_t sin = (op_reads(d->op) && in) ? ia + lo * esz : 0;
    const uint64_t sout = (op_writes(d->op) && out) ? oa + lo * esz : 0;
    uint64_t saux = 0;
    if (d->aux && op_has_result(d->op)) saux = d->aux + 8ull * j;
    if (d->aux && d->op == LK_OP_AXPY_F32) saux = d->aux + lo * esz;
    post_cmd(c, mbs[j], t, LKW_TO_WORK + d->op, hi - lo, sin, sout, saux, static_cast<uint32_t>(d->a),
             static_cast<uint32_t>(d->b), d->alpha, j, d->flags);
  }
  cs.posted = t;
  *ticket = t;
  return LK_OK;
}

int lk_submit_batch(lk_ctx *c, uint32_t cluster, const lk_tile *tiles, uint32_t n_tiles, int64_t *partials,
                    uint64_t *ticket) {
  if (!c || !ticket) return fail(LK_EINVAL, "NULL argument");
  if (c->state != RUNNING) return fail(LK_ESTATE, "context is not running");
  if (cluster >= c->n_clusters) return fail(LK_EINVAL, "cluster %u of %u", cluster, c->n_clusters);
  const uint64_t ta = reinterpret_cast<uint64_t>(tiles), pa = reinterpret_cast<uint64_t>(partials);
  if (n_tiles && (!tiles || (ta & 15u) || !partials || (pa & 7u)))
    return fail(LK_EINVAL, "tiles must be 16-byte aligned and partials 8-byte aligned, non-NULL");
  if ((ta | pa) >> LKW_TAG_SHIFT) return fail(LK_EINVAL, "pointer outside the 48-bit address range");
  ClusterSeq &cs = c->seqs[cluster];
  const uint64_t t = cs.posted + 1;
  if (t - cs.consumed > c->depth) return fail(LK_EAGAIN, "ring full (depth %u)", c->depth);
  const std::vector<uint32_t> &mbs = c->cluster_mbox[cluster];
  for (uint32_t mb : mbs)
    if (exited_code(worker_code(c, mb))) return fail(LK_ESTATE, "worker of mailbox %u has exited", mb);
  const size_t slot = static_cast<size_t>(cluster) * c->depth + ring_slot(c, t);
  uint64_t &base = c->batch_base[slot];
  const uint64_t counter = reinterpret_cast<uint64_t>(c->d_batch_counters) + slot * 128;
  for (uint32_t j = 0; j < mbs.size(); ++j)
    post_cmd(c, mbs[j], t, LKW_TO_WORK + LK_OP_BATCH, n_tiles, ta, pa, counter, static_cast<uint32_t>(base),
             static_cast<uint32_t>(base >> 32), 0.f, j);
  base += static_cast<uint64_t>(n_tiles) + mbs.size();
  cs.posted = t;
  *ticket = t;
  return LK_OK;
}

int lk_batch_plan(const lk_desc *items, const uint64_t *in_addr, const uint64_t *out_addr, uint32_t count,
                  uint64_t tile_elems, lk_tile *tiles, uint32_t *tile_item, uint32_t cap, uint32_t *n_tiles) {
  if (!n_tiles || (count && (!items || !in_addr || !out_addr))) return fail(LK_EINVAL, "NULL argument");
  if (tile_elems == 0 || tile_elems % 256 || tile_elems > (1ull << 31)) return fail(LK_EINVAL, "tile_elems must be a positive multiple of 256 up to 2^31");
  uint64_t need = 0;
  for (uint32_t i = 0; i < count; ++i) {
    const lk_desc &d = items[i];
    if (d.op >= LK_OP_COUNT || d.op == LK_OP_BATCH) return fail(LK_EINVAL, "item %u: op %u cannot be tiled", i, d.op);
    if (d.flags || d.reserved) return fail(LK_EINVAL, "item %u: tiles take no descriptor flags", i);
    if ((in_addr[i] | out_addr[i]) & 3u) return fail(LK_EINVAL, "item %u: pointers must be 4-byte aligned", i);
    need += d.n == 0 ? 1 : (d.n + tile_elems - 1) / tile_elems;
  }
  *n_tiles = static_cast<uint32_t>(need);
  if (need > cap || need > 0xffffffffull) return fail(LK_EINVAL, "%llu tiles exceed cap %u", static_cast<unsigned long long>(need), cap);
  uint32_t k = 0;
  for (uint32_t i = 0; i < count; ++i) {
    const lk_desc &d = items[i];
    uint32_t bbits;
    memcpy(&bbits, &d.alpha, 4);
    if (d.op != LK_OP_SAXPY_F32 && d.op != LK_OP_AXPY_F32) bbits = static_cast<uint32_t>(d.b);
    if (d.op == LK_OP_AXPY_F32 && (d.n && (!d.aux || (d.aux & 3u))))
      return fail(LK_EINVAL, "item %u: AXPY_F32 needs y (aux) 4-byte aligned", i);
    const uint64_t parts = d.n == 0 ? 1 : (d.n + tile_elems - 1) / tile_elems;
    for (uint64_t p = 0; p < parts; ++p) {
      const uint64_t lo = p * tile_elems, len = std::min<uint64_t>(tile_elems, d.n - std::min(d.n, lo));
      lk_tile &tl = tiles[k];
      tl.in = op_reads(d.op) ? in_addr[i] + lo * 4 : 0;
      tl.out = op_writes(d.op) ? out_addr[i] + lo * 4 : 0;
      tl.in2 = d.op == LK_OP_AXPY_F32 ? d.aux + lo * 4 : 0;
      tl.reserved = 0;
      tl.n = static_cast<uint32_t>(len);
      tl.op = d.op;
      tl.a = d.a;
      tl.b = bbits;
      if (tile_item) tile_item[k] = i;
      ++k;
    }
  }
  return LK_OK;
}

// Member records of one ticket, folded as they are read.
struct Fold {
  int64_t sum = 0;
  uint64_t pmin = ~0ull, pmax = 0, dmin = ~0ull, dmax = 0;
  bool fault = false;
  void add(const Status &s) {
    fault |= s.code == LKW_FROM_ERROR;
    sum += s.partial;
    pmin = std::min(pmin, s.t_pick);
    pmax = std::max(pmax, s.t_pick);
    dmin = std::min(dmin, s.t_done);
    dmax = std::max(dmax, s.t_done);
  }
};

// Releases a ticket whose every member has finished and reports it.
static int release_ticket(ClusterSeq &cs, uint64_t t, const Fold &f, lk_completion *info) {
  cs.consumed = t;
  if (info) {
    info->result = f.sum;
    info->t_pick_min = f.pmin;
    info->t_pick_max = f.pmax;
    info->t_done_min = f.dmin;
    info->t_done_max = f.dmax;
  }
  if (f.fault) return fail(LK_EFAULT, "a worker rejected ticket %llu", static_cast<unsigned long long>(t));
  return LK_OK;
}

// Checks shared by the Wait calls; on success *cs is the cluster's sequence state.
static int wait_args(lk_ctx *c, uint32_t cluster, uint64_t t, ClusterSeq **cs) {
  if (!c) return fail(LK_EINVAL, "NULL context");
  if (c->state != RUNNING) return fail(LK_ESTATE, "context is not running");
  if (cluster >= c->n_clusters) return fail(LK_EINVAL, "cluster %u of %u", cluster, c->n_clusters);
  *cs = &c->seqs[cluster];
  if (t == 0 || t > (*cs)->posted) return fail(LK_EINVAL, "ticket %llu was not posted", static_cast<unsigned long long>(t));
  if (t <= (*cs)->consumed) return fail(LK_EINVAL, "ticket %llu already released", static_cast<unsigned long long>(t));
  return LK_OK;
}

static int wait_impl(lk_ctx *c, uint32_t cluster, uint64_t t, int64_t timeout_ns, lk_completion *info) {
  ClusterSeq *cs = nullptr;
  if (const int rc = wait_args(c, cluster, t, &cs)) return rc;
  const bool bounded = timeout_ns >= 0;
  const auto deadline = bounded ? clk::now() + std::chrono::nanoseconds(timeout_ns) : clk::time_point::max();
  Fold f;
  for (uint32_t mb : c->cluster_mbox[cluster]) {
    const lkw_status *rec = slot_status(c, mb, t);
    uint32_t spins = 0;
    Status s;
    while (!read_status(rec, t, &s)) {
      if ((++spins & 255u) == 0) {
        if (bounded && clk::now() > deadline) return fail(LK_ETIMEDOUT, "ticket %llu not finished", static_cast<unsigned long long>(t));
        if (exited_code(worker_code(c, mb))) {
          if (read_status(rec, t, &s)) break;
          return fail(LK_ESTATE, "worker of mailbox %u exited before finishing ticket %llu", mb,
                      static_cast<unsigned long long>(t));
        }
      }
      _mm_pause();
    }
    f.add(s);
  }
  return release_ticket(*cs, t, f, info);
}

int lk_try_wait(lk_ctx *c, uint32_t cluster, uint64_t t, lk_completion *info) {
  ClusterSeq *cs = nullptr;
  if (const int rc = wait_args(c, cluster, t, &cs)) return rc;
  Fold f;
  for (uint32_t mb : c->cluster_mbox[cluster]) {
    const lkw_status *rec = slot_status(c, mb, t);
    Status s;
    if (!read_status(rec, t, &s)) {
      if (!exited_code(worker_code(c, mb))) return LK_EAGAIN;  // not yet: nothing changes
      if (!read_status(rec, t, &s))
        return fail(LK_ESTATE, "worker of mailbox %u exited before finishing ticket %llu", mb,
                    static_cast<unsigned long long>(t));
    }
    f.add(s);
  }
  return release_ticket(*cs, t, f, info);
}

int lk_wait(lk_ctx *c, uint32_t cluster, uint64_t ticket, int64_t timeout_ns, int64_t *result) {
  lk_completion info;
  const int rc = wait_impl(c, cluster, ticket, timeout_ns, &info);
  if (rc == LK_OK && result) *result = info.result;
  return rc;
}

int lk_wait_info(lk_ctx *c, uint32_t cluster, uint64_t ticket, int64_t timeout_ns, lk_completion *out) {
  if (!out) return fail(LK_EINVAL, "out is NULL");
  return wait_impl(c, cluster, ticket, timeout_ns, out);
}

int lk_poll(lk_ctx *c, uint32_t cluster, uint64_t t, int *done) {
  if (!c || !done) return fail(LK_EINVAL, "NULL argument");
  if (c->state != RUNNING) return fail(LK_ESTATE, "context is not running");
  if (cluster >= c->n_clusters) return fail(LK_EINVAL, "cluster %u of %u", cluster, c->n_clusters);
  const ClusterSeq &cs = c->seqs[cluster];
  if (t == 0 || t > cs.posted) return fail(LK_EINVAL, "ticket was not posted");
  if (t <= cs.consumed) {
    *done = 1;
    return LK_OK;
  }
  int all = 1;
  for (uint32_t mb : c->cluster_mbox[cluster]) {
    if (!read_status(slot_status(c, mb, t), t, nullptr)) {
      all = 0;
      break;
    }
  }
  *done = all;
  return LK_OK;
}

__attribute__((target("prfchw"))) int lk_prefetch(lk_ctx *c, uint32_t cluster, uint64_t t) {
  if (!c) return fail(LK_EINVAL, "NULL context");
  if (c->state != RUNNING) return fail(LK_ESTATE, "context is not running");
  if (cluster >= c->n_clusters) return fail(LK_EINVAL, "cluster %u of %u", cluster, c->n_clusters);
  const ClusterSeq &cs = c->seqs[cluster];
  const bool pending = t > cs.consumed && t <= cs.posted;
  const uint64_t next = cs.posted + 1;
  for (uint32_t mb : c->cluster_mbox[cluster]) {
    if (pending) __builtin_prefetch(slot_status(c, mb, t), 0, 3);
    __builtin_prefetch(slot_cmd(c, mb, next), 1, 3);  // will be written
  }
  return LK_OK;
}

int lk_dispose(lk_ctx *c) {
  if (!c) return fail(LK_EINVAL, "NULL context");
  if (c->state == DISPOSED) return LK_OK;
  if (c->state == POISONED) {
    if (!c->kernel_launched || join_kernel(c, 0.5)) {
      release_gpu(c);
      c->state = DISPOSED;
      return LK_OK;
    }
    return fail(LK_ETIMEDOUT, "context poisoned: persistent kernel still running");
  }
  const auto t0 = clk::now();
  const uint32_t idle_ms = c->cfg.idle_timeout_ms ? c->cfg.idle_timeout_ms : 10000u;
  // Let every posted item finish (bounded), then post THREAD_EXIT behind it.
  const auto drain_deadline = t0 + std::chrono::seconds(10);
  for (uint32_t k = 0; k < c->n_clusters; ++k) {
    const uint64_t t = c->seqs[k].posted;
    for (uint32_t mb : c->cluster_mbox[k]) {
      if (t > c->seqs[k].consumed) {
        const lkw_status *st = slot_status(c, mb, t);
        while (!read_status(st, t, nullptr)) {
          if (exited_code(worker_code(c, mb)) || clk::now() > drain_deadline) break;
          _mm_pause();
        }
      }
      if (!exited_code(worker_code(c, mb))) post_cmd(c, mb, t + 1, LKW_TO_EXIT, 0, 0, 0, 0, 0, 0, 0.f, 0);
    }
    c->seqs[k].consumed = t;
  }
  if (!join_kernel(c, 5.0 + idle_ms / 1000.0)) {
    c->state = POISONED;
    return fail(LK_ETIMEDOUT, "persistent kernel did not end after EXIT (context poisoned)");
  }
  c->kernel_ms = c->wq ? c->wq->kernel_ms() : 0.0;
  if (c->d_log && c->log_cap) {
    c->host_log.resize(static_cast<size_t>(c->n_workers) * c->log_cap);
    std::string err;
    if (lkbe::device_to_host(c->host_log.data(), c->d_log, sizeof(lkw_log) * c->host_log.size(), &err) != LK_OK)
      c->host_log.clear();
  }
  // Worker records survive for lk_get_info: keep a copy of the exit codes and the span
  // from the first boot to the last exit on the device wall clock.
  uint32_t exited = 0;
  uint64_t boot_min = ~0ull, exit_max = 0;
  for (uint32_t m = 0; m < c->n_workers; ++m) {
    exited += exited_code(worker_code(c, m));
    boot_min = std::min(boot_min, __atomic_load_n(&c->wrec[m].t_boot, __ATOMIC_RELAXED));
    exit_max = std::max(exit_max, __atomic_load_n(&c->wrec[m].t_exit, __ATOMIC_RELAXED));
  }
  if (exit_max > boot_min) c->device_span_ms = static_cast<double>(exit_max - boot_min) * 1e3 / static_cast<double>(c->wall_hz);
  c->exited_at_dispose = exited;
  release_gpu(c);
  c->state = DISPOSED;
  c->dispose_ms = std::chrono::duration<double, std::milli>(clk::now() - t0).count();
  return LK_OK;
}

int lk_free(lk_ctx *c) {
  if (!c) return LK_OK;
  int rc = LK_OK;
  if (c->state != DISPOSED) rc = lk_dispose(c);
  if (c->state != DISPOSED) return rc;  // poisoned: keep the object so nothing dangles
  delete c;
  return LK_OK;
}

int lk_get_info(lk_ctx *c, lk_info *info) {
  if (!c || !info) return fail(LK_EINVAL, "NULL argument");
  memset(info, 0, sizeof *info);
  info->n_workers = c->n_workers;
  info->n_clusters = c->n_clusters;
  info->queue_depth = c->depth;
  info->threads_per_worker = c->threads;
  info->cu_count = c->cu_count;
  info->xcd_count = c->xcd_count;
  info->state = c->state;
  if (c->state == RUNNING) {
    for (uint32_t m = 0; m < c->n_workers; ++m) info->workers_exited += exited_code(worker_code(c, m));
  } else {
    info->workers_exited = c->exited_at_dispose;
  }
  info->wall_clock_hz = c->wall_hz;
  info->init_ms = c->init_ms;
  info->dispose_ms = c->dispose_ms;
  info->kernel_ms = c->kernel_ms;
  info->device_span_ms = c->device_span_ms;
  info->workers_per_cu = c->per_cu;
  info->max_workers_on_a_cu = c->max_on_a_cu;
  info->pin_capacity = c->pin_bytes;
  info->xcd_mask = c->xcd_mask;
  return LK_OK;
}

int lk_topology(lk_ctx *c, uint32_t w, uint32_t *xcc, uint32_t *se, uint32_t *sh, uint32_t *cu) {
  if (!c) return fail(LK_EINVAL, "NULL context");
  if (w >= c->workers.size()) return fail(LK_EINVAL, "worker %u of %zu", w, c->workers.size());
  const WorkerInfo &x = c->workers[w];
  if (xcc) *xcc = x.xcc;
  if (se) *se = x.se;
  if (sh) *sh = x.sh;
  if (cu) *cu = x.cu;
  return LK_OK;
}

int lk_cluster_members(lk_ctx *c, uint32_t cluster, uint32_t *workers, uint32_t cap, uint32_t *count) {
  if (!c || !count) return fail(LK_EINVAL, "NULL argument");
  if (cluster >= c->n_clusters) return fail(LK_EINVAL, "cluster %u of %u", cluster, c->n_clusters);
  const auto &m = c->clusters[cluster];
  *count = static_cast<uint32_t>(m.size());
  if (workers)
    for (uint32_t i = 0; i < m.size() && i < cap; ++i) workers[i] = m[i];
  return LK_OK;
}

int lk_read_log(lk_ctx *c, uint32_t w, lk_log_entry *out, uint32_t cap, uint32_t *count) {
  if (!c || !count) return fail(LK_EINVAL, "NULL argument");
  *count = 0;
  if (c->state != DISPOSED) return fail(LK_ESTATE, "the log is available after lk_dispose");
  if (w >= c->workers.size()) return fail(LK_EINVAL, "worker %u of %zu", w, c->workers.size());
  if (c->host_log.empty()) return LK_OK;
  const uint32_t mb = c->workers[w].mailbox;
  const lkw_log *L = c->host_log.data() + static_cast<size_t>(mb) * c->log_cap;
  // Entries are written at (seq-1) % cap; collect the valid ones, oldest first.
  std::vector<lkw_log> v;
  for (uint32_t i = 0; i < c->log_cap; ++i)
    if (L[i].seq) v.push_back(L[i]);
  std::sort(v.begin(), v.end(), [](const lkw_log &a, const lkw_log &b) { return a.seq < b.seq; });
  const size_t skip = v.size() > cap ? v.size() - cap : 0;
  uint32_t n = 0;
  for (size_t i = skip; i < v.size(); ++i) {
    if (out) {
      out[n].seq = v[i].seq;
      out[n].code = v[i].code;
      out[n].worker = static_cast<uint16_t>(w);
      out[n].xcc = v[i].xcc;
      out[n].hwid = v[i].hwid;
      out[n].t_pick = v[i].t_pick;
      out[n].t_done = v[i].t_done;
    }
    ++n;
  }
  *count = n;
  return LK_OK;
}

}  // extern "C"
