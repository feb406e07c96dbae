/*
 * lk_serve.cpp -- continuous-batching serving loop over the persistent workers
 * (include/lk_serve.h).
 */
#include "lk_serve.h"

#include <immintrin.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <atomic>
#include <chrono>
#include <deque>
#include <thread>
#include <vector>

#include "lk.h"
#include "lk_affinity.hpp"
#include "lk_arena.hpp"
#include "lk_error.h"

namespace {

// Record the detail of a rejected call for lk_last_error and return the code.
int sfail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int sfail(int code, const char *fmt, ...) {
  char buf[256];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  lkh::set_last_error(buf);
  return code;
}

using clk = std::chrono::steady_clock;
using lksrv::Arena;

constexpr uint64_t kGranule = Arena::kGranule;  // bytes; output buffers start 256-byte aligned

bool op_allowed(uint32_t op) {
  return op == LK_OP_AFFINE_SUM_I32 || op == LK_OP_SUM_I32_I64 || op == LK_OP_AXPY_F32 || op == LK_OP_COPY_F32;
}
uint64_t out_bytes(const lks_request &r) { return r.op == LK_OP_SUM_I32_I64 ? 0 : r.n * 4; }

struct Tile {
  uint64_t req;  // request index
  uint64_t lo, len;
};

struct Active {
  uint64_t remaining = 0;
  int64_t sum = 0;
  uint64_t out = 0;
};

struct Posted {
  uint64_t ticket;
  uint64_t req;
  clk::time_point t_post;
};

}  // namespace

extern "C" int lks_run(lk_ctx *c, const lks_config *cfg, const lks_request *reqs, uint64_t count, lks_outcome *out,
                       lks_stats *stats) {
  if (!c || !cfg || (!reqs && count) || (!out && count)) return sfail(LK_EINVAL, "lks_run: NULL argument");
  lk_info info;
  if (lk_get_info(c, &info) != LK_OK || info.state != 0) return sfail(LK_ESTATE, "lks_run: context is not running");
  if (info.n_clusters != info.n_workers)
    return sfail(LK_EINVAL, "lks_run: needs one cluster per worker (%u clusters, %u workers)", info.n_clusters,
                 info.n_workers);
  const uint32_t T = cfg->threads;
  if (T == 0 || T > 64 || T > info.n_workers)
    return sfail(LK_EINVAL, "lks_run: %u scheduler threads: need 1..64 and at most the %u workers", T, info.n_workers);
  if (cfg->tile_elems == 0 || cfg->tile_elems % 256 || cfg->tile_elems > (1ull << 31))
    return sfail(LK_EINVAL, "lks_run: tile_elems must be a positive multiple of 256 up to 2^31");
  if ((cfg->arena & (kGranule - 1)) || (cfg->arena_bytes && !cfg->arena))
    return sfail(LK_EINVAL, "lks_run: arena must be non-NULL and %llu-byte aligned",
                 static_cast<unsigned long long>(kGranule));
  for (uint64_t i = 0; i < count; ++i) {
    const lks_request &r = reqs[i];
    if (!op_allowed(r.op) || ((r.in | r.in2) & 3u) || (r.n && !r.in) || (r.op == LK_OP_AXPY_F32 && r.n && !r.in2))
      return sfail(LK_EINVAL, "lks_run: request %llu: op %u not served or pointer NULL or not 4-byte aligned",
                   static_cast<unsigned long long>(i), r.op);
    if (i && r.arrival_us < reqs[i - 1].arrival_us)
      return sfail(LK_EINVAL, "lks_run: request %llu arrives before the one preceding it",
                   static_cast<unsigned long long>(i));
    out[i] = lks_outcome{0, 0, -1.0, -1.0, LK_OK, 0};
  }
  const uint64_t slice = cfg->arena_bytes / T / kGranule * kGranule;
  const uint32_t depth = info.queue_depth;
  std::atomic<int> error{LK_OK};
  std::vector<uint64_t> tiles_done(T, 0), deferred(T, 0), peak(T, 0), tiles_posted(T, 0), tiles_drained(T, 0);
  std::atomic<uint32_t> undrained{0};
  // The arrival clock starts only once every shard has built its tables (they are sized
  // by the trace and page-faulted in while being filled), so that set-up is not charged
  // to the first requests as queueing.
  std::atomic<uint32_t> ready{0};
  std::atomic<int64_t> t0_ns{0};
  clk::time_point t0;
  auto us_since = [&](clk::time_point t) { return std::chrono::duration<double, std::micro>(t - t0).count(); };

  // Scheduler threads on distinct CPUs when there are enough (the caller's thread keeps one).
  const bool pin = T < lkaff::allowed_cpus().size();
  auto shard = [&](uint32_t s) {
    if (pin) lkaff::pin_to_allowed_cpu(s);
    Arena arena(cfg->arena + s * slice, slice);
    std::vector<uint32_t> workers;
    for (uint32_t w = s; w < info.n_workers; w += T) workers.push_back(w);
    std::vector<std::deque<Posted>> posted(workers.size());
    std::vector<uint64_t> mine;  // request indices of this shard, arrival order
    for (uint64_t i = s; i < count; i += T) mine.push_back(i);
    size_t next_arrival = 0;
    std::deque<uint64_t> waiting;   // arrived, not admitted
    std::deque<Tile> queue;         // tiles of admitted requests, admission order
    // State of this shard's requests, indexed by i / T (request i belongs to shard i % T).
    std::vector<Active> act(mine.size());
    uint64_t n_active = 0;
    uint64_t finished = 0;
    uint64_t last_deferred = ~0ull;  // the waiting head already counted as deferred
    uint32_t rr = 0;
    ready.fetch_add(1, std::memory_order_acq_rel);
    while (t0_ns.load(std::memory_order_acquire) == 0) _mm_pause();
    // One pass of the scheduler: arrivals, admission, completions, dispatch.  Returns
    // LK_OK or the error that ends this shard; every way out of the loop below reaches the
    // drain after it.
    auto step = [&]() -> int {
      const auto now = clk::now();
      const double now_us = us_since(now);
      // 1. arrivals
      while (next_arrival < mine.size() && reqs[mine[next_arrival]].arrival_us <= now_us) waiting.push_back(mine[next_arrival++]);
      // 2. admission, first come first served, against the shard's memory budget
      while (!waiting.empty()) {
        const uint64_t i = waiting.front();
        const lks_request &r = reqs[i];
        uint64_t addr = 0;
        const uint64_t need = out_bytes(r);
        if (need) {
          if (Arena::round(need) > arena.size()) return LK_EINVAL;  // can never fit
          if (!arena.alloc(need, &addr)) {
            // Nothing in flight in this shard means nothing will ever be freed: the
            // budget is exhausted for good (possible only with `retain`).
            if (n_active == 0) return LK_EINVAL;
            if (i != last_deferred) {
              ++deferred[s];
              last_deferred = i;
            }
            break;
          }
        }
        waiting.pop_front();
        const uint64_t nt = r.n == 0 ? 1 : (r.n + cfg->tile_elems - 1) / cfg->tile_elems;
        Active a;
        a.remaining = nt;
        a.out = addr;
        act[i / T] = a;
        ++n_active;
        out[i].admit_us = now_us;
        out[i].out = addr;
        out[i].tiles = static_cast<uint32_t>(nt);
        for (uint64_t k = 0; k < nt; ++k) {
          const uint64_t lo = k * cfg->tile_elems;
          queue.push_back(Tile{i, lo, std::min(cfg->tile_elems, r.n - std::min(r.n, lo))});
        }
      }
      // 3. completions
      for (size_t w = 0; w < workers.size(); ++w) {
        auto &pq = posted[w];
        while (!pq.empty()) {
          lk_completion ci;
          const int rc = lk_try_wait(c, workers[w], pq.front().ticket, &ci);
          if (rc == LK_EAGAIN) {
            if (cfg->timeout_ns >= 0 && now - pq.front().t_post > std::chrono::nanoseconds(cfg->timeout_ns))
              return LK_ETIMEDOUT;
            break;
          }
          if (rc) return rc;
          const int64_t part = ci.result;
          const uint64_t i = pq.front().req;
          pq.pop_front();
          ++tiles_done[s];
          Active &a = act[i / T];
          a.sum += part;
          if (--a.remaining == 0) {
            out[i].result = a.sum;
            out[i].done_us = us_since(clk::now());
            if (!cfg->retain && a.out) arena.release(a.out, out_bytes(reqs[i]));
            --n_active;
            ++finished;
          }
        }
      }
      // 4. dispatch, breadth first: every idle worker gets a tile, then every worker holding
      // one gets a second, and so on up to the ring depth, so that a new request's tiles
      // do not queue behind earlier tiles while one of the shard's workers is idle.
      for (uint32_t level = 0; level < depth && !queue.empty(); ++level) {
        for (size_t k = 0; k < workers.size() && !queue.empty(); ++k) {
          const size_t w = (rr + k) % workers.size();
          if (posted[w].size() != level) continue;
          const Tile tl = queue.front();
          const lks_request &r = reqs[tl.req];
          lk_desc d{};
          d.op = r.op;
          d.n = tl.len;
          d.a = r.a;
          d.b = r.b;
          d.alpha = r.alpha;
          d.aux = r.op == LK_OP_AXPY_F32 ? r.in2 + tl.lo * 4 : 0;
          const uint64_t in = r.in + tl.lo * 4;
          const uint64_t ob = act[tl.req / T].out;
          const uint64_t o = ob ? ob + tl.lo * 4 : 0;
          uint64_t t;
          const int rc = lk_submit(c, workers[w], &d, reinterpret_cast<const void *>(in), reinterpret_cast<void *>(o), &t);
          if (rc == LK_EAGAIN) continue;
          if (rc) return rc;
          posted[w].push_back(Posted{t, tl.req, clk::now()});
          ++tiles_posted[s];
          queue.pop_front();
        }
      }
      rr = workers.empty() ? 0 : (rr + 1) % workers.size();
      return LK_OK;
    };
    while (finished < mine.size() && error.load(std::memory_order_relaxed) == LK_OK) {
      const int rc = step();
      if (rc != LK_OK) {
        int expected = LK_OK;
        error.compare_exchange_strong(expected, rc);
        break;
      }
      _mm_pause();
    }
    peak[s] = arena.peak();
    // After an error (this shard's or another's) tiles may still be posted: wait for each
    // of them, so that no tile of this run still reads or writes memory when lks_run
    // returns.  A tile that does not finish within the drain deadline is left to the
    // caller-visible fallback below (disposing the context).
    const int64_t drain_ns = cfg->timeout_ns >= 0 ? std::max<int64_t>(cfg->timeout_ns, 1000000000ll) : -1;
    for (size_t w = 0; w < workers.size(); ++w)
      for (const Posted &p : posted[w]) {
        const int rc = lk_wait(c, workers[w], p.ticket, drain_ns, nullptr);
        if (rc == LK_ETIMEDOUT) {
          undrained.fetch_add(1, std::memory_order_relaxed);
          break;  // later tickets of this worker run after it: none of them finished either
        }
        if (rc == LK_OK) ++tiles_drained[s];
      }
  };
  std::vector<std::thread> th;
  for (uint32_t s = 0; s < T; ++s) th.emplace_back(shard, s);
  while (ready.load(std::memory_order_acquire) < T) std::this_thread::yield();
  t0 = clk::now() + std::chrono::milliseconds(2);
  t0_ns.store(std::max<int64_t>(1, t0.time_since_epoch().count()), std::memory_order_release);
  for (auto &t : th) t.join();
  int rc = error.load();
  if (undrained.load() != 0) {
    // A posted tile did not finish within the drain deadline and may still touch the
    // arena or the request buffers: dispose the context, which either ends the workers
    // (every tile done) or leaves the context poisoned (lk_get_info state 2), telling the
    // caller that this memory may still be written.
    (void)lk_dispose(c);
    if (rc == LK_OK) rc = LK_ETIMEDOUT;
  }
  if (stats) {
    double last = 0;
    for (uint64_t i = 0; i < count; ++i) last = std::max(last, out[i].done_us);
    stats->elapsed_s = (last - (count ? reqs[0].arrival_us : 0.0)) * 1e-6;
    stats->tiles = stats->deferred = stats->peak_bytes = stats->posted = stats->drained = 0;
    for (uint32_t s = 0; s < T; ++s) {
      stats->tiles += tiles_done[s];
      stats->deferred += deferred[s];
      stats->peak_bytes += peak[s];
      stats->posted += tiles_posted[s];
      stats->drained += tiles_drained[s];
    }
  }
  if (rc)
    for (uint64_t i = 0; i < count; ++i)
      if (out[i].done_us < 0) out[i].status = rc;
  return rc;
}
