/*
 * lk_bench.cpp -- native timed runners, per-launch baselines and probes (include/lk_bench.h).
 */
#include <hip/hip_runtime_api.h>
#include <immintrin.h>
#include <x86intrin.h>

#include <pthread.h>
#include <sched.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "lk.h"
#include "lk_affinity.hpp"
#include "lk_bench.h"
#include "lk_device.h"
#include "lk_error.h"
#include "lk_scratch.h"

namespace {

using clk = std::chrono::steady_clock;

inline double us_between(clk::time_point a, clk::time_point b) {
  return std::chrono::duration<double, std::micro>(b - a).count();
}

int bfail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int bfail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  lkh::set_last_error(buf);
  fprintf(stderr, "lk_bench: %s\n", buf);
  return code;
}

inline uint64_t load_acquire(const uint64_t *p) { return __atomic_load_n(p, __ATOMIC_ACQUIRE); }

using lkaff::allowed_cpus;
using lkaff::pin_to_allowed_cpu;

lk_desc to_desc(const lkb_item &it) {
  lk_desc d{};
  d.op = it.op;
  d.n = it.n;
  d.a = it.a;
  d.b = it.b;
  d.alpha = it.alpha;
  d.aux = it.op == LK_OP_AXPY_F32 ? it.in2 : 0;
  d.flags = it.flags;
  return d;
}

bool valid_item(const lkb_item &it) {
  if (it.op >= LK_OP_COUNT) return false;
  if ((it.in | it.out | it.in2) & 3u) return false;
  return true;
}

// Host-coherent scratch for the per-launch paths: completion words and partials.
struct CoherentRegion {
  void *p = nullptr;
  ~CoherentRegion() {
    if (p) (void)hipHostFree(p);
  }
  hipError_t alloc(size_t bytes) {
    hipError_t e = hipHostMalloc(&p, bytes, hipHostMallocCoherent | hipHostMallocMapped | hipHostMallocPortable);
    if (e == hipSuccess) memset(p, 0, bytes);
    return e;
  }
};

struct DeviceBuf {
  void *p = nullptr;
  ~DeviceBuf() {
    if (p) (void)hipFree(p);
  }
};

// One single-node graph of the item kernel, parameters updated per item.
struct ItemGraph {
  hipGraph_t g = nullptr;
  hipGraphExec_t exec = nullptr;
  hipGraphNode_t node = nullptr;
  lkd::ItemArgs args{};
  void *kparams[1] = {&args};
  hipKernelNodeParams np{};
  uint32_t k = 1, threads = 256;
  ItemGraph() = default;
  ItemGraph(const ItemGraph &) = delete;
  ItemGraph &operator=(const ItemGraph &) = delete;
  ~ItemGraph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (g) (void)hipGraphDestroy(g);
  }
  hipError_t build(uint32_t k_, uint32_t threads_) {
    k = k_;
    threads = threads_;
    hipError_t e = hipGraphCreate(&g, 0);
    if (e != hipSuccess) return e;
    np.func = const_cast<void *>(lkd::item_kernel());
    np.gridDim = dim3(k);
    np.blockDim = dim3(threads);
    np.sharedMemBytes = 0;
    np.kernelParams = kparams;
    np.extra = nullptr;
    args.k = k;
    e = hipGraphAddKernelNode(&node, g, nullptr, 0, &np);
    if (e != hipSuccess) return e;
    return hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
  }
  hipError_t launch(const lkd::ItemArgs &a, hipStream_t s) {
    args = a;
    np.kernelParams = kparams;
    hipError_t e = hipGraphExecKernelNodeSetParams(exec, node, &np);
    if (e != hipSuccess) return e;
    return hipGraphLaunch(exec, s);
  }
};

lkd::ItemArgs item_args(const lkb_item &it, uint32_t k) {
  lkd::ItemArgs a{};
  a.op = it.op;
  a.k = k;
  a.n = it.n;
  a.in = reinterpret_cast<const void *>(it.in);
  a.out = reinterpret_cast<void *>(it.out);
  a.in2 = reinterpret_cast<const void *>(it.in2);
  a.a = static_cast<uint32_t>(it.a);
  a.b = static_cast<uint32_t>(it.b);
  a.alpha = it.alpha;
  return a;
}

// LKB_GRAPH_CHAIN form of lkb_launch_lanes: each lane's items captured once, in order, as
// one hipGraph on the lane's stream; the timed region launches every lane's graph and
// waits until every stream is idle.
int graph_chain_lanes(uint32_t n_lanes, const lkb_item *items, uint64_t items_per_lane,
                      std::vector<hipStream_t> &streams, uint32_t threads, int64_t *results, double *lat_us,
                      double *elapsed_s) {
  const uint64_t total = static_cast<uint64_t>(n_lanes) * items_per_lane;
  CoherentRegion parts;  // one int64 partial per item
  hipError_t e = parts.alloc(8ull * (total ? total : 1));
  if (e != hipSuccess) return bfail(LK_EHIP, "hipHostMalloc: %s", hipGetErrorString(e));
  std::vector<hipGraphExec_t> execs(n_lanes, nullptr);
  int rc = LK_OK;
  for (uint32_t l = 0; l < n_lanes && rc == LK_OK; ++l) {
    hipStream_t s = streams[l % streams.size()];
    if ((e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal)) != hipSuccess) {
      rc = bfail(LK_EHIP, "begin capture: %s", hipGetErrorString(e));
      break;
    }
    hipError_t le = hipSuccess;
    for (uint64_t k = 0; k < items_per_lane && le == hipSuccess; ++k) {
      const uint64_t idx = static_cast<uint64_t>(l) * items_per_lane + k;
      lkd::ItemArgs a = item_args(items[idx], 1);
      a.partials = static_cast<int64_t *>(parts.p) + idx;
      le = lkd::launch_item(a, threads, s);
    }
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(s, &g);
    if (le != hipSuccess || e != hipSuccess) {
      rc = bfail(LK_EHIP, "capture: %s", hipGetErrorString(le != hipSuccess ? le : e));
    } else if ((e = hipGraphInstantiate(&execs[l], g, nullptr, nullptr, 0)) != hipSuccess) {
      rc = bfail(LK_EHIP, "instantiate: %s", hipGetErrorString(e));
    }
    if (g) (void)hipGraphDestroy(g);
  }
  if (rc == LK_OK) {
    const auto start = clk::now();
    for (uint32_t l = 0; l < n_lanes && rc == LK_OK; ++l)
      if ((e = hipGraphLaunch(execs[l], streams[l % streams.size()])) != hipSuccess)
        rc = bfail(LK_EHIP, "graph launch: %s", hipGetErrorString(e));
    for (hipStream_t s : streams)
      if ((e = hipStreamSynchronize(s)) != hipSuccess && rc == LK_OK)
        rc = bfail(LK_EHIP, "synchronize: %s", hipGetErrorString(e));
    if (elapsed_s) *elapsed_s = std::chrono::duration<double>(clk::now() - start).count();
  }
  for (hipGraphExec_t x : execs)
    if (x) (void)hipGraphExecDestroy(x);
  if (rc != LK_OK) return rc;
  for (uint64_t i = 0; i < total; ++i) {
    if (results) results[i] = __atomic_load_n(static_cast<int64_t *>(parts.p) + i, __ATOMIC_RELAXED);
    if (lat_us) lat_us[i] = 0.0;
  }
  return LK_OK;
}

}  // namespace

extern "C" {

int lkb_serial(lk_ctx *c, uint32_t cluster, const lkb_item *items, uint64_t count, int64_t timeout_ns,
               int64_t *results, double *lat_us, double *trigger_us, lk_completion *info) {
  if (!c || (!items && count)) return bfail(LK_EINVAL, "NULL argument");
  for (uint64_t i = 0; i < count; ++i) {
    const lk_desc d = to_desc(items[i]);
    uint64_t t = 0;
    const auto t0 = clk::now();
    int rc = lk_submit(c, cluster, &d, reinterpret_cast<const void *>(items[i].in),
                       reinterpret_cast<void *>(items[i].out), &t);
    const auto t1 = clk::now();
    if (rc) return rc;
    lk_completion ci;
    rc = lk_wait_info(c, cluster, t, timeout_ns, &ci);
    const auto t2 = clk::now();
    if (rc) return rc;
    if (results) results[i] = ci.result;
    if (lat_us) lat_us[i] = us_between(t0, t2);
    if (trigger_us) trigger_us[i] = us_between(t0, t1);
    if (info) info[i] = ci;
  }
  return LK_OK;
}

int lkb_lanes(lk_ctx *c, const uint32_t *lane_cluster, uint32_t n_lanes, const lkb_item *items,
              uint64_t items_per_lane, uint32_t in_flight, uint32_t n_threads, int64_t timeout_ns, int64_t *results,
              double *lat_us, double *elapsed_s, lk_completion *info) {
  if (!c || !lane_cluster || (!items && items_per_lane)) return bfail(LK_EINVAL, "NULL argument");
  if (n_threads == 0 || n_threads > 256 || in_flight == 0 || in_flight > LK_MAX_DEPTH)
    return bfail(LK_EINVAL, "n_threads 1..256 and in_flight 1..%u", LK_MAX_DEPTH);
  lk_info inf;
  lk_get_info(c, &inf);
  if (in_flight > inf.queue_depth) return bfail(LK_EINVAL, "in_flight %u > queue depth %u", in_flight, inf.queue_depth);
  if (n_threads > n_lanes) n_threads = n_lanes ? n_lanes : 1;
  std::atomic<int> error{0};
  std::atomic<bool> stop{false};
  const auto start = clk::now();
  // Each host thread owns a fixed set of lanes (one producer per mailbox).  Per lane and
  // per sweep: first collect every finished ticket, then refill up to in_flight, so a
  // lane is re-armed as soon as its completion is seen.  Threads are pinned to distinct
  // allowed CPUs when there are enough of them (the caller's thread only waits to join
  // them, so it needs no CPU of its own).
  const bool pin = n_threads <= allowed_cpus().size();
  auto worker = [&](uint32_t tix) {
    if (pin) pin_to_allowed_cpu(tix);
    // Submit times of the items in flight, in a ring of in_flight entries (item k in
    // entry k % in_flight), so the per-item bookkeeping stays in the thread's caches.
    struct Lane {
      uint32_t id, cluster;
      uint64_t next = 0, done = 0;
      uint64_t first_ticket = 0;  // ticket of item 0
      clk::time_point t_sub[LK_MAX_DEPTH];
    };
    std::vector<Lane> lanes;
    for (uint32_t l = tix; l < n_lanes; l += n_threads) {
      Lane L{};
      L.id = l;
      L.cluster = lane_cluster[l];
      lanes.push_back(L);
    }
    // The next items' descriptors and output slots are fetched a few items ahead: a thread
    // serves many lanes, each with its own streams through these arrays.
    constexpr uint64_t kItemsAhead = 2;
    auto prefetch_item = [&](const Lane &L, uint64_t k) {
      if (k >= items_per_lane) return;
      const uint64_t idx = static_cast<uint64_t>(L.id) * items_per_lane + k;
      __builtin_prefetch(items + idx, 0, 3);
      if (results) __builtin_prefetch(results + idx, 1, 3);
      if (lat_us) __builtin_prefetch(lat_us + idx, 1, 3);
      if (info) __builtin_prefetch(info + idx, 1, 3);
    };
    auto fail_all = [&](int rc) {
      error.store(rc);
      stop.store(true);
    };
    uint64_t remaining = lanes.size() * items_per_lane;
    const size_t nl = lanes.size();
    constexpr size_t kAhead = 6;  // lanes between a prefetch and its use (about one memory miss)
    while (remaining && !stop.load(std::memory_order_relaxed)) {
      for (size_t li = 0; li < nl; ++li) {
        Lane &L = lanes[li];
        if (nl > kAhead) {
          const Lane &A = lanes[(li + kAhead) % nl];
          (void)lk_prefetch(c, A.cluster, A.done < A.next ? A.first_ticket + A.done : 0);
        }
        while (L.done < L.next) {
          const uint64_t t = L.first_ticket + L.done;
          lk_completion ci;
          const int rc = lk_try_wait(c, L.cluster, t, &ci);
          if (rc == LK_EAGAIN) {
            if (timeout_ns >= 0 &&
                clk::now() - L.t_sub[L.done % in_flight] > std::chrono::nanoseconds(timeout_ns))
              return fail_all(LK_ETIMEDOUT);
            break;
          }
          if (rc) return fail_all(rc);
          const auto now = clk::now();
          const uint64_t idx = static_cast<uint64_t>(L.id) * items_per_lane + L.done;
          if (results) results[idx] = ci.result;
          if (lat_us) lat_us[idx] = us_between(L.t_sub[L.done % in_flight], now);
          if (info) info[idx] = ci;
          ++L.done;
          --remaining;
        }
        while (L.next < items_per_lane && L.next - L.done < in_flight) {
          const lkb_item &it = items[static_cast<uint64_t>(L.id) * items_per_lane + L.next];
          const lk_desc d = to_desc(it);
          uint64_t t;
          const auto ts = clk::now();
          const int rc = lk_submit(c, L.cluster, &d, reinterpret_cast<const void *>(it.in),
                                   reinterpret_cast<void *>(it.out), &t);
          if (rc == LK_EAGAIN) break;
          if (rc) return fail_all(rc);
          L.t_sub[L.next % in_flight] = ts;
          if (L.next == 0) L.first_ticket = t;
          ++L.next;
          prefetch_item(L, L.next + kItemsAhead - 1);
        }
      }
      _mm_pause();
    }
  };
  std::vector<std::thread> th;
  for (uint32_t t = 0; t < n_threads; ++t) th.emplace_back(worker, t);
  for (auto &t : th) t.join();
  if (elapsed_s) *elapsed_s = std::chrono::duration<double>(clk::now() - start).count();
  const int rc = error.load();
  if (rc) return bfail(rc, "lanes run failed: %s", lk_strerror(rc));
  return LK_OK;
}

int lkb_isolation(lk_ctx *c, uint32_t crit_cluster, const lkb_item *crit, uint64_t periods, int64_t period_ns,
                  const uint32_t *bg_clusters, uint32_t n_bg, const lkb_item *bg, int64_t *results, double *lat_us,
                  double *late_us, lk_completion *info, uint64_t *bg_done, double *elapsed_s) {
  if (!c || (!crit && periods) || (!bg && n_bg) || (!bg_clusters && n_bg)) return bfail(LK_EINVAL, "NULL argument");
  if (period_ns <= 0 || n_bg > 64) return bfail(LK_EINVAL, "period_ns > 0 and n_bg <= 64");
  for (uint32_t i = 0; i < n_bg; ++i)
    if (bg_clusters[i] == crit_cluster) return bfail(LK_EINVAL, "background cluster %u is the critical one", crit_cluster);
  std::atomic<bool> stop{false};
  std::atomic<int> bg_error{0};
  std::vector<uint64_t> counts(n_bg, 0);
  const size_t ncpu = allowed_cpus().size();
  // Background streams: one host thread per interfering cluster re-posts its item as soon
  // as the previous one completes.
  auto bg_worker = [&](uint32_t i) {
    if (ncpu > n_bg + 1) pin_to_allowed_cpu(i);  // the last allowed CPU stays the critical thread's
    const lk_desc d = to_desc(bg[i]);
    while (!stop.load(std::memory_order_relaxed)) {
      uint64_t t;
      int rc = lk_submit(c, bg_clusters[i], &d, reinterpret_cast<const void *>(bg[i].in),
                         reinterpret_cast<void *>(bg[i].out), &t);
      if (rc == LK_OK) rc = lk_wait(c, bg_clusters[i], t, 30000000000ll, nullptr);
      if (rc) {
        bg_error.store(rc);
        return;
      }
      ++counts[i];
    }
  };
  std::vector<std::thread> th;
  for (uint32_t i = 0; i < n_bg; ++i) th.emplace_back(bg_worker, i);

  // Critical stream on the calling thread, pinned to the last allowed CPU for the run:
  // release k happens at t0 + k * period (busy-wait), then submit and wait.
  cpu_set_t old_set;
  const bool pinned = ncpu > n_bg + 1 && pthread_getaffinity_np(pthread_self(), sizeof old_set, &old_set) == 0;
  if (pinned) pin_to_allowed_cpu(ncpu - 1);
  int rc = LK_OK;
  const auto start = clk::now();
  const auto t0 = start + std::chrono::milliseconds(20);  // let the interference ramp up
  for (uint64_t k = 0; k < periods && rc == LK_OK; ++k) {
    const auto release = t0 + std::chrono::nanoseconds(period_ns * static_cast<int64_t>(k));
    while (clk::now() < release) _mm_pause();
    const auto ts = clk::now();
    const lk_desc d = to_desc(crit[k]);
    uint64_t t;
    rc = lk_submit(c, crit_cluster, &d, reinterpret_cast<const void *>(crit[k].in), reinterpret_cast<void *>(crit[k].out), &t);
    if (rc) break;
    lk_completion ci;
    rc = lk_wait_info(c, crit_cluster, t, 5000000000ll, &ci);
    const auto te = clk::now();
    if (rc) break;
    if (results) results[k] = ci.result;
    if (lat_us) lat_us[k] = us_between(release, te);
    if (late_us) late_us[k] = us_between(release, ts);
    if (info) info[k] = ci;
    if (bg_error.load()) rc = bg_error.load();
  }
  if (elapsed_s) *elapsed_s = std::chrono::duration<double>(clk::now() - start).count();
  stop.store(true);
  for (auto &t : th) t.join();
  if (pinned) pthread_setaffinity_np(pthread_self(), sizeof old_set, &old_set);
  for (uint32_t i = 0; i < n_bg; ++i)
    if (bg_done) bg_done[i] = counts[i];
  if (!rc) rc = bg_error.load();
  if (rc) return bfail(rc, "isolation run failed: %s (%s)", lk_strerror(rc), lk_last_error());
  return LK_OK;
}

int lkb_replay(int device, uint32_t n_workers, uint32_t spin_iters, uint32_t runs, double *lk_us, double *hip_us,
               uint64_t *lk_cycles, uint64_t *hip_cycles, int64_t *results) {
  if (runs == 0 || n_workers == 0 || n_workers > LK_MAX_WORKERS) return bfail(LK_EINVAL, "bad runs/n_workers");
  hipError_t e = hipSetDevice(device);
  if (e != hipSuccess) return bfail(LK_EHIP, "hipSetDevice: %s", hipGetErrorString(e));
  lkb_item spin_item{};
  spin_item.op = LK_OP_SPIN;
  spin_item.a = static_cast<int32_t>(spin_iters);
  const lk_desc d = to_desc(spin_item);
  auto record = [](double *us, uint64_t *cy, uint32_t r, int phase, clk::time_point a, clk::time_point b, uint64_t ca,
                   uint64_t cb) {
    if (us) us[r * 4 + phase] = us_between(a, b);
    if (cy) cy[r * 4 + phase] = cb - ca;
  };
  for (uint32_t r = 0; r < runs; ++r) {
    // ---- persistent path: Init, Trigger, Wait, Dispose
    lk_config cfg;
    lk_config_default(&cfg);
    cfg.device = device;
    cfg.n_workers = n_workers;
    cfg.cluster_policy = LK_CLUSTERS_ONE;  // one Trigger reaches every worker
    cfg.idle_timeout_ms = 20000;
    lk_ctx *c = nullptr;
    auto a = clk::now();
    uint64_t ca = __rdtsc();
    int rc = lk_init(&cfg, &c);
    uint64_t cb = __rdtsc();
    auto b = clk::now();
    if (rc) return bfail(rc, "replay lk_init: %s", lk_last_error());
    record(lk_us, lk_cycles, r, 0, a, b, ca, cb);
    uint64_t t;
    a = clk::now();
    ca = __rdtsc();
    rc = lk_submit(c, 0, &d, nullptr, nullptr, &t);
    cb = __rdtsc();
    b = clk::now();
    record(lk_us, lk_cycles, r, 1, a, b, ca, cb);
    if (rc == LK_OK) {
      int64_t res = 0;
      a = clk::now();
      ca = __rdtsc();
      rc = lk_wait(c, 0, t, 10000000000ll, &res);
      cb = __rdtsc();
      b = clk::now();
      record(lk_us, lk_cycles, r, 2, a, b, ca, cb);
      if (results) results[2ull * r] = res;
    }
    a = clk::now();
    ca = __rdtsc();
    const int rc2 = lk_dispose(c);
    cb = __rdtsc();
    b = clk::now();
    record(lk_us, lk_cycles, r, 3, a, b, ca, cb);
    lk_free(c);
    if (rc || rc2) return bfail(rc ? rc : rc2, "replay persistent run %u: %s", r, lk_last_error());

    // ---- per-launch path: Alloc, Spawn, Wait, Dispose
    void *buf = nullptr;
    hipStream_t s = nullptr;
    a = clk::now();
    ca = __rdtsc();
    const size_t buf_bytes = std::max<size_t>(4096, 8ull * n_workers);  // one int64 result per workgroup
    e = hipMalloc(&buf, buf_bytes);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    cb = __rdtsc();
    b = clk::now();
    if (e != hipSuccess) return bfail(LK_EHIP, "replay alloc: %s", hipGetErrorString(e));
    record(hip_us, hip_cycles, r, 0, a, b, ca, cb);
    lkd::ItemArgs ia = item_args(spin_item, n_workers);
    ia.aux = static_cast<int64_t *>(buf);
    a = clk::now();
    ca = __rdtsc();
    e = lkd::launch_item(ia, 256, s);
    cb = __rdtsc();
    b = clk::now();
    record(hip_us, hip_cycles, r, 1, a, b, ca, cb);
    if (e != hipSuccess) return bfail(LK_EHIP, "replay spawn: %s", hipGetErrorString(e));
    a = clk::now();
    ca = __rdtsc();
    e = hipStreamSynchronize(s);
    cb = __rdtsc();
    b = clk::now();
    record(hip_us, hip_cycles, r, 2, a, b, ca, cb);
    if (e != hipSuccess) return bfail(LK_EHIP, "replay wait: %s", hipGetErrorString(e));
    if (results) {  // the item's result, summed over its workgroups (not timed)
      std::vector<int64_t> parts(n_workers);
      e = hipMemcpy(parts.data(), buf, 8ull * n_workers, hipMemcpyDeviceToHost);
      if (e != hipSuccess) return bfail(LK_EHIP, "replay result copy: %s", hipGetErrorString(e));
      int64_t sum = 0;
      for (int64_t v : parts) sum += v;
      results[2ull * r + 1] = sum;
    }
    a = clk::now();
    ca = __rdtsc();
    (void)hipStreamDestroy(s);
    e = hipFree(buf);
    cb = __rdtsc();
    b = clk::now();
    record(hip_us, hip_cycles, r, 3, a, b, ca, cb);
    if (e != hipSuccess) return bfail(LK_EHIP, "replay dispose: %s", hipGetErrorString(e));
  }
  return LK_OK;
}

int lkb_batch(lk_ctx *c, uint32_t cluster, const lk_tile *tiles, uint32_t n_tiles, int64_t *partials, uint32_t reps,
              int64_t timeout_ns, double *makespan_us, lk_completion *info) {
  if (!c || reps == 0) return bfail(LK_EINVAL, "NULL context or reps == 0");
  for (uint32_t r = 0; r < reps; ++r) {
    uint64_t t;
    const auto t0 = clk::now();
    int rc = lk_submit_batch(c, cluster, tiles, n_tiles, partials, &t);
    if (rc) return rc;
    lk_completion ci;
    rc = lk_wait_info(c, cluster, t, timeout_ns, &ci);
    const auto t1 = clk::now();
    if (rc) return rc;
    if (ci.result != static_cast<int64_t>(n_tiles))
      return bfail(LK_EFAULT, "batch executed %lld tiles of %u", static_cast<long long>(ci.result), n_tiles);
    if (makespan_us) makespan_us[r] = us_between(t0, t1);
    if (info) info[r] = ci;
  }
  return LK_OK;
}

int lkb_launch_burst(int device, const lkb_item *items, uint32_t count, uint64_t elems_per_wg, uint32_t threads,
                     uint32_t mode, uint32_t reps, double *makespan_us) {
  if ((!items && count) || reps == 0 || elems_per_wg == 0 || threads < 64 || threads > 1024 || threads % 64)
    return bfail(LK_EINVAL, "bad burst arguments");
  for (uint32_t i = 0; i < count; ++i)
    if (!valid_item(items[i]) || items[i].op == LK_OP_BATCH) return bfail(LK_EINVAL, "item %u invalid", i);
  hipError_t e = hipSetDevice(device);
  if (e != hipSuccess) return bfail(LK_EHIP, "hipSetDevice: %s", hipGetErrorString(e));
  hipStream_t s;
  if ((e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking)) != hipSuccess) return bfail(LK_EHIP, "stream: %s", hipGetErrorString(e));
  DeviceBuf counters;  // one per item (grids of more than one workgroup)
  int rc = LK_OK;
  if ((e = hipMalloc(&counters.p, 64ull * (count ? count : 1))) != hipSuccess ||
      (e = hipMemset(counters.p, 0, 64ull * (count ? count : 1))) != hipSuccess)
    rc = bfail(LK_EHIP, "counters: %s", hipGetErrorString(e));
  auto launch_all = [&]() -> hipError_t {
    for (uint32_t i = 0; i < count; ++i) {
      const uint64_t k64 = (items[i].n + elems_per_wg - 1) / elems_per_wg;
      const uint32_t k = static_cast<uint32_t>(k64 < 1 ? 1 : (k64 > 4096 ? 4096 : k64));
      lkd::ItemArgs a = item_args(items[i], k);
      a.counter = reinterpret_cast<uint32_t *>(static_cast<char *>(counters.p) + 64ull * i);
      const hipError_t le = lkd::launch_item(a, threads, s);
      if (le != hipSuccess) return le;
    }
    return hipSuccess;
  };
  hipGraph_t g = nullptr;
  hipGraphExec_t ge = nullptr;
  const bool use_graph = mode & LKB_USE_GRAPH;
  if (rc == LK_OK && use_graph) {
    // Capture the burst once (not timed), instantiate, then time graph launches.
    if ((e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal)) != hipSuccess)
      rc = bfail(LK_EHIP, "begin capture: %s", hipGetErrorString(e));
    if (rc == LK_OK) {
      const hipError_t le = launch_all();
      e = hipStreamEndCapture(s, &g);
      if (le != hipSuccess || e != hipSuccess) rc = bfail(LK_EHIP, "capture: %s", hipGetErrorString(le != hipSuccess ? le : e));
    }
    if (rc == LK_OK && (e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0)) != hipSuccess)
      rc = bfail(LK_EHIP, "instantiate: %s", hipGetErrorString(e));
  }
  for (uint32_t r = 0; rc == LK_OK && r < reps; ++r) {
    const auto t0 = clk::now();
    e = use_graph ? hipGraphLaunch(ge, s) : launch_all();
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    const auto t1 = clk::now();
    if (e != hipSuccess) rc = bfail(LK_EHIP, "burst: %s", hipGetErrorString(e));
    else if (makespan_us) makespan_us[r] = us_between(t0, t1);
  }
  (void)hipStreamSynchronize(s);
  if (ge) (void)hipGraphExecDestroy(ge);
  if (g) (void)hipGraphDestroy(g);
  (void)hipStreamDestroy(s);
  return rc;
}

int lkb_launch_serial(int device, uint32_t k, uint32_t threads, const lkb_item *items, uint64_t count, uint32_t mode,
                      int64_t *results, double *lat_us, double *launch_us) {
  if (!items && count) return bfail(LK_EINVAL, "NULL items");
  if (k == 0 || k > 4096 || threads < 64 || threads > 1024 || threads % 64) return bfail(LK_EINVAL, "bad k/threads");
  for (uint64_t i = 0; i < count; ++i)
    if (!valid_item(items[i])) return bfail(LK_EINVAL, "item %llu invalid", static_cast<unsigned long long>(i));
  hipError_t e = hipSetDevice(device);
  if (e != hipSuccess) return bfail(LK_EHIP, "hipSetDevice: %s", hipGetErrorString(e));
  hipStream_t s;
  if ((e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking)) != hipSuccess)
    return bfail(LK_EHIP, "hipStreamCreate: %s", hipGetErrorString(e));
  CoherentRegion reg;
  DeviceBuf counter;
  int rc = LK_OK;
  ItemGraph graph;
  const bool flag = mode & LKB_COMPLETE_FLAG, use_graph = mode & LKB_USE_GRAPH;
  if ((e = reg.alloc(4096 + 8ull * k)) != hipSuccess) {
    rc = bfail(LK_EHIP, "hipHostMalloc: %s", hipGetErrorString(e));
  } else if ((e = hipMalloc(&counter.p, 256)) != hipSuccess || (e = hipMemset(counter.p, 0, 256)) != hipSuccess) {
    rc = bfail(LK_EHIP, "counter: %s", hipGetErrorString(e));
  } else if (use_graph && (e = graph.build(k, threads)) != hipSuccess) {
    rc = bfail(LK_EHIP, "graph build: %s", hipGetErrorString(e));
  }
  uint64_t *done_word = static_cast<uint64_t *>(reg.p);
  int64_t *partials = reinterpret_cast<int64_t *>(static_cast<char *>(reg.p) + 4096);
  for (uint64_t i = 0; rc == LK_OK && i < count; ++i) {
    lkd::ItemArgs a = item_args(items[i], k);
    a.partials = partials;
    a.counter = static_cast<uint32_t *>(counter.p);
    if (flag) {
      a.done_word = done_word;
      a.done_value = i + 1;
    }
    const auto t0 = clk::now();
    e = use_graph ? graph.launch(a, s) : lkd::launch_item(a, threads, s);
    const auto t1 = clk::now();
    if (e != hipSuccess) {
      rc = bfail(LK_EHIP, "launch: %s", hipGetErrorString(e));
      break;
    }
    if (flag) {
      const auto deadline = t0 + std::chrono::seconds(10);
      uint32_t spins = 0;
      while (load_acquire(done_word) != i + 1) {
        if ((++spins & 1023u) == 0 && clk::now() > deadline) {
          rc = bfail(LK_ETIMEDOUT, "item %llu: completion word not seen", static_cast<unsigned long long>(i));
          break;
        }
        _mm_pause();
      }
    } else {
      e = hipStreamSynchronize(s);
      if (e != hipSuccess) rc = bfail(LK_EHIP, "hipStreamSynchronize: %s", hipGetErrorString(e));
    }
    const auto t2 = clk::now();
    if (rc) break;
    int64_t sum = 0;
    for (uint32_t j = 0; j < k; ++j) sum += __atomic_load_n(partials + j, __ATOMIC_RELAXED);
    if (results) results[i] = sum;
    if (lat_us) lat_us[i] = us_between(t0, t2);
    if (launch_us) launch_us[i] = us_between(t0, t1);
  }
  (void)hipStreamSynchronize(s);
  (void)hipStreamDestroy(s);
  return rc;
}

int lkb_launch_serial_static(int device, uint32_t k, uint32_t threads, const lkb_item *items, uint64_t count,
                             int64_t *results, double *lat_us, double *launch_us) {
  if (!items && count) return bfail(LK_EINVAL, "NULL items");
  if (k == 0 || k > lkd::kStaticMaxK)
    return bfail(LK_EINVAL, "k = %u workgroups: the static partial-result array holds 1..%u", k, lkd::kStaticMaxK);
  if (threads < 64 || threads > 1024 || threads % 64) return bfail(LK_EINVAL, "bad threads");
  for (uint64_t i = 0; i < count; ++i)
    if (!valid_item(items[i])) return bfail(LK_EINVAL, "item %llu invalid", static_cast<unsigned long long>(i));
  hipError_t e = hipSetDevice(device);
  if (e != hipSuccess) return bfail(LK_EHIP, "hipSetDevice: %s", hipGetErrorString(e));
  int64_t *partials = nullptr;
  if ((e = lkd::static_partials(device, &partials)) != hipSuccess)
    return bfail(LK_EHIP, "static scratch address: %s", hipGetErrorString(e));
  // The null stream, so that nothing is created; every entry 0..k-1 of the array is
  // written by workgroup j of each launch before it is read, so nothing is cleared.
  hipStream_t s = nullptr;
  constexpr uint32_t kChunk = 512;  // partials read back in chunks through a stack buffer
  int64_t buf[kChunk];
  for (uint64_t i = 0; i < count; ++i) {
    lkd::ItemArgs a = item_args(items[i], k);
    a.partials = partials;
    const auto t0 = clk::now();
    e = lkd::launch_item(a, threads, s);
    const auto t1 = clk::now();
    if (e != hipSuccess) return bfail(LK_EHIP, "launch: %s", hipGetErrorString(e));
    if ((e = hipStreamSynchronize(s)) != hipSuccess)
      return bfail(LK_EHIP, "hipStreamSynchronize: %s", hipGetErrorString(e));
    const auto t2 = clk::now();
    int64_t sum = 0;
    for (uint32_t j0 = 0; j0 < k; j0 += kChunk) {
      const uint32_t m = std::min(kChunk, k - j0);
      if ((e = hipMemcpy(buf, partials + j0, 8ull * m, hipMemcpyDeviceToHost)) != hipSuccess)
        return bfail(LK_EHIP, "partials copy: %s", hipGetErrorString(e));
      for (uint32_t j = 0; j < m; ++j) sum += buf[j];
    }
    if (results) results[i] = sum;
    if (lat_us) lat_us[i] = us_between(t0, t2);
    if (launch_us) launch_us[i] = us_between(t0, t1);
  }
  return LK_OK;
}

int lkb_launch_lanes(int device, uint32_t n_lanes, const lkb_item *items, uint64_t items_per_lane, uint32_t n_streams,
                     uint32_t n_threads, uint32_t threads, uint32_t mode, int64_t *results, double *lat_us,
                     double *elapsed_s) {
  if (!items && items_per_lane) return bfail(LK_EINVAL, "NULL items");
  if (n_lanes == 0 || n_lanes > 65536 || n_streams == 0 || n_streams > 64 || n_threads == 0 || n_threads > 256 ||
      threads < 64 || threads > 1024 || threads % 64)
    return bfail(LK_EINVAL, "bad lanes/streams/threads");
  for (uint64_t i = 0; i < static_cast<uint64_t>(n_lanes) * items_per_lane; ++i)
    if (!valid_item(items[i])) return bfail(LK_EINVAL, "item %llu invalid", static_cast<unsigned long long>(i));
  hipError_t e = hipSetDevice(device);
  if (e != hipSuccess) return bfail(LK_EHIP, "hipSetDevice: %s", hipGetErrorString(e));
  if (n_threads > n_lanes) n_threads = n_lanes;
  std::vector<hipStream_t> streams(n_streams, nullptr);
  int rc = LK_OK;
  for (auto &s : streams)
    if (rc == LK_OK && (e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking)) != hipSuccess)
      rc = bfail(LK_EHIP, "hipStreamCreate: %s", hipGetErrorString(e));
  CoherentRegion reg;  // per lane: done word + partial, 64 bytes apart
  if (rc == LK_OK && (e = reg.alloc(64ull * n_lanes)) != hipSuccess)
    rc = bfail(LK_EHIP, "hipHostMalloc: %s", hipGetErrorString(e));
  if (mode & LKB_GRAPH_CHAIN) {
    if (rc == LK_OK) rc = graph_chain_lanes(n_lanes, items, items_per_lane, streams, threads, results, lat_us, elapsed_s);
    for (auto &s : streams)
      if (s) (void)hipStreamDestroy(s);
    return rc;
  }
  std::vector<ItemGraph> graphs(mode & LKB_USE_GRAPH ? n_lanes : 0);
  for (auto &g : graphs)
    if (rc == LK_OK && (e = g.build(1, threads)) != hipSuccess) rc = bfail(LK_EHIP, "graph build: %s", hipGetErrorString(e));
  std::atomic<int> error{rc};
  std::atomic<bool> stop{rc != LK_OK};
  const auto start = clk::now();
  const bool pin = n_threads < allowed_cpus().size();  // as in lkb_lanes
  auto worker = [&](uint32_t tix) {
    if (pin) pin_to_allowed_cpu(tix);
    struct Lane {
      uint32_t id;
      uint64_t next = 0;
      bool busy = false;
      clk::time_point t0{};
    };
    std::vector<Lane> lanes;
    for (uint32_t l = tix; l < n_lanes; l += n_threads) {
      Lane L{};
      L.id = l;
      lanes.push_back(L);
    }
    uint64_t remaining = lanes.size() * items_per_lane;
    while (remaining && !stop.load(std::memory_order_relaxed)) {
      for (Lane &L : lanes) {
        char *slot = static_cast<char *>(reg.p) + 64ull * L.id;
        uint64_t *done_word = reinterpret_cast<uint64_t *>(slot);
        int64_t *partial = reinterpret_cast<int64_t *>(slot + 8);
        if (L.busy) {
          if (load_acquire(done_word) != L.next + 1) {
            if (clk::now() - L.t0 > std::chrono::seconds(10)) {
              error.store(LK_ETIMEDOUT);
              stop.store(true);
              return;
            }
            continue;
          }
          const auto now = clk::now();
          const uint64_t idx = static_cast<uint64_t>(L.id) * items_per_lane + L.next;
          if (results) results[idx] = __atomic_load_n(partial, __ATOMIC_RELAXED);
          if (lat_us) lat_us[idx] = us_between(L.t0, now);
          L.busy = false;
          ++L.next;
          --remaining;
        }
        if (!L.busy && L.next < items_per_lane) {
          const lkb_item &it = items[static_cast<uint64_t>(L.id) * items_per_lane + L.next];
          lkd::ItemArgs a = item_args(it, 1);
          a.partials = partial;
          a.done_word = done_word;
          a.done_value = L.next + 1;
          hipStream_t s = streams[L.id % n_streams];
          L.t0 = clk::now();
          const hipError_t le = graphs.empty() ? lkd::launch_item(a, threads, s) : graphs[L.id].launch(a, s);
          if (le != hipSuccess) {
            error.store(LK_EHIP);
            stop.store(true);
            return;
          }
          L.busy = true;
        }
      }
      _mm_pause();
    }
  };
  std::vector<std::thread> th;
  if (rc == LK_OK)
    for (uint32_t t = 0; t < n_threads; ++t) th.emplace_back(worker, t);
  for (auto &t : th) t.join();
  if (elapsed_s) *elapsed_s = std::chrono::duration<double>(clk::now() - start).count();
  for (auto &s : streams)
    if (s) {
      (void)hipStreamSynchronize(s);
      (void)hipStreamDestroy(s);
    }
  graphs.clear();
  rc = error.load();
  if (rc) return bfail(rc, "launch lanes failed: %s", lk_strerror(rc));
  return LK_OK;
}

int lkb_pingpong(int device, uint32_t workers, uint64_t iters, uint32_t poll_sleep, int spread, double *rtt_us) {
  if (workers == 0 || workers > 1024 || iters == 0 || iters > 10000000ull || poll_sleep > 127)
    return bfail(LK_EINVAL, "bad workers/iters/poll_sleep");
  hipError_t e = hipSetDevice(device);
  if (e != hipSuccess) return bfail(LK_EHIP, "hipSetDevice: %s", hipGetErrorString(e));
  hipDeviceProp_t prop;
  if ((e = hipGetDeviceProperties(&prop, device)) != hipSuccess) return bfail(LK_EHIP, "props: %s", hipGetErrorString(e));
  if (spread && workers > static_cast<uint32_t>(prop.multiProcessorCount))
    return bfail(LK_EINVAL, "spread pingpong needs workers <= CU count");
  int wc_khz = 100000;
  (void)hipDeviceGetAttribute(&wc_khz, hipDeviceAttributeWallClockRate, device);
  const uint32_t stride = 16;  // one 128-byte line per worker and direction
  CoherentRegion reg;
  if ((e = reg.alloc(2ull * workers * stride * 8)) != hipSuccess) return bfail(LK_EHIP, "hipHostMalloc: %s", hipGetErrorString(e));
  uint64_t *h2d = static_cast<uint64_t *>(reg.p);
  uint64_t *d2h = h2d + static_cast<uint64_t>(workers) * stride;
  DeviceBuf status;
  if ((e = hipMalloc(&status.p, 4ull * workers)) != hipSuccess || (e = hipMemset(status.p, 0, 4ull * workers)) != hipSuccess)
    return bfail(LK_EHIP, "status: %s", hipGetErrorString(e));
  hipStream_t s;
  if ((e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking)) != hipSuccess) return bfail(LK_EHIP, "stream: %s", hipGetErrorString(e));
  // Device deadline: generous bound on the whole run (50 us per echo + 5 s).
  const double run_s = 5.0 + 50e-6 * static_cast<double>(iters) * workers;
  const uint64_t deadline_ticks = static_cast<uint64_t>(run_s * wc_khz * 1000.0);
  e = lkd::launch_pingpong(h2d, d2h, stride, workers, iters, deadline_ticks, poll_sleep, static_cast<uint32_t *>(status.p),
                           spread != 0, s);
  int rc = LK_OK;
  if (e != hipSuccess) rc = bfail(LK_EHIP, "launch pingpong: %s", hipGetErrorString(e));
  for (uint64_t i = 1; rc == LK_OK && i <= iters; ++i) {
    for (uint32_t w = 0; w < workers; ++w) {
      uint64_t *in = h2d + static_cast<uint64_t>(w) * stride;
      uint64_t *out = d2h + static_cast<uint64_t>(w) * stride;
      const auto t0 = clk::now();
      __atomic_store_n(in, i, __ATOMIC_RELEASE);
      uint32_t spins = 0;
      while (load_acquire(out) < i) {
        if ((++spins & 1023u) == 0 && clk::now() - t0 > std::chrono::seconds(2)) {
          rc = bfail(LK_ETIMEDOUT, "pingpong worker %u iteration %llu: no echo", w, static_cast<unsigned long long>(i));
          break;
        }
        _mm_pause();
      }
      if (rc) break;
      if (rtt_us) rtt_us[static_cast<uint64_t>(w) * iters + (i - 1)] = us_between(t0, clk::now());
    }
  }
  if (rc) {  // release every worker so the kernel ends before its deadline
    for (uint32_t w = 0; w < workers; ++w) __atomic_store_n(h2d + static_cast<uint64_t>(w) * stride, iters, __ATOMIC_RELEASE);
  }
  (void)hipStreamSynchronize(s);
  (void)hipStreamDestroy(s);
  return rc;
}

int lkb_copy(int device, const void *src, void *dst, uint64_t bytes, uint32_t grid, uint32_t threads,
             uint32_t unroll, uint32_t policy, uint32_t reps, double *ms_avg, double *gbps) {
  if (!src || !dst || bytes % 16 || (reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) % 16 ||
      grid == 0 || grid > (1u << 20) || reps == 0)
    return bfail(LK_EINVAL, "bad copy arguments");
  if (threads < 64 || threads > 1024 || threads % 64 || (unroll != 4 && unroll != 8 && unroll != 16))
    return bfail(LK_EINVAL, "copy: threads 64..1024 in whole waves, unroll 4, 8 or 16");
  if (policy > LKB_COPY_SYSTEM || (policy == LKB_COPY_SYSTEM && bytes >= (1ull << 31)))
    return bfail(LK_EINVAL, "copy: unknown store policy, or written-through stores over 2 GiB or more");
  hipError_t e = hipSetDevice(device);
  if (e != hipSuccess) return bfail(LK_EHIP, "hipSetDevice: %s", hipGetErrorString(e));
  hipStream_t s;
  if ((e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking)) != hipSuccess) return bfail(LK_EHIP, "stream: %s", hipGetErrorString(e));
  hipEvent_t a, b;
  (void)hipEventCreate(&a);
  (void)hipEventCreate(&b);
  int rc = LK_OK;
  auto launch = [&]() { return lkd::launch_copy_probe(src, dst, bytes, grid, threads, unroll, policy, s); };
  // one untimed warm-up
  if ((e = launch()) != hipSuccess) rc = bfail(LK_EHIP, "copy: %s", hipGetErrorString(e));
  (void)hipEventRecord(a, s);
  for (uint32_t r = 0; rc == LK_OK && r < reps; ++r)
    if ((e = launch()) != hipSuccess) rc = bfail(LK_EHIP, "copy: %s", hipGetErrorString(e));
  (void)hipEventRecord(b, s);
  (void)hipStreamSynchronize(s);
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, a, b);
  if (ms_avg) *ms_avg = ms / reps;
  if (gbps) *gbps = ms > 0 ? 2.0 * bytes * reps / (ms * 1e-3) / 1e9 : 0.0;
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  (void)hipStreamDestroy(s);
  return rc;
}

}  // extern "C"
