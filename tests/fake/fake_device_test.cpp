// Host-logic scenarios of the dispatch library (lk_host.cpp, lk_serve.cpp) against the
// fake device of lk_backend_fake.cpp.  Built with -fsanitize=thread by
// tests/test_fake_device.py; prints "OK <scenario>" per scenario and exits 0, or prints
// the failed check and exits 1.
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <atomic>
#include <chrono>
#include <cmath>
#include <random>
#include <thread>
#include <vector>

#include "lk.h"
#include "lk_serve.h"

extern "C" void lkfake_freeze(int mailbox);

#define CHECK(c)                                                                            \
  do {                                                                                      \
    if (!(c)) {                                                                             \
      fprintf(stderr, "%s: check failed at line %d: %s (%s)\n", g_case, __LINE__, #c, lk_last_error()); \
      exit(1);                                                                              \
    }                                                                                       \
  } while (0)

static const char *g_case = "";

static lk_ctx *open_ctx(uint32_t n_workers, uint32_t depth, uint32_t policy, uint32_t idle_ms = 20000,
                        uint32_t log_cap = 0) {
  lk_config cfg;
  lk_config_default(&cfg);
  cfg.n_workers = n_workers;
  cfg.queue_depth = depth;
  cfg.cluster_policy = policy;
  cfg.idle_timeout_ms = idle_ms;
  cfg.log_capacity = log_cap;
  lk_ctx *c = nullptr;
  CHECK(lk_init(&cfg, &c) == LK_OK && c);
  return c;
}

static void affine_ref(const int32_t *x, uint64_t n, int32_t a, int32_t b, int32_t *y, int64_t *s) {
  int64_t acc = 0;
  for (uint64_t i = 0; i < n; ++i) {
    y[i] = static_cast<int32_t>(static_cast<uint32_t>(a) * static_cast<uint32_t>(x[i]) + static_cast<uint32_t>(b));
    acc += y[i];
  }
  *s = acc;
}

static lk_desc desc(uint32_t op, uint64_t n, int32_t a = 0, int32_t b = 0, float alpha = 0.f, uint64_t aux = 0) {
  lk_desc d;
  memset(&d, 0, sizeof d);
  d.op = op;
  d.n = n;
  d.a = a;
  d.b = b;
  d.alpha = alpha;
  d.aux = aux;
  return d;
}

// T2.6: one worker, 1000 submit-then-wait items, exact, FIFO in the log.
static void single_worker_1000() {
  g_case = "single_worker_1000";
  lk_ctx *c = open_ctx(1, 1, LK_CLUSTERS_PER_WORKER, 20000, 1024);
  const uint64_t n = 257;
  std::mt19937 rng(1);
  std::vector<int32_t> x(n), y(n), yr(n);
  for (int it = 0; it < 1000; ++it) {
    for (auto &v : x) v = static_cast<int32_t>(rng());
    const int32_t a = static_cast<int32_t>(rng()), b = static_cast<int32_t>(rng());
    lk_desc d = desc(LK_OP_AFFINE_SUM_I32, n, a, b);
    uint64_t t;
    CHECK(lk_submit(c, 0, &d, x.data(), y.data(), &t) == LK_OK);
    CHECK(t == static_cast<uint64_t>(it) + 1);
    int64_t s = 0, sr = 0;
    CHECK(lk_wait(c, 0, t, 5000000000ll, &s) == LK_OK);
    affine_ref(x.data(), n, a, b, yr.data(), &sr);
    CHECK(s == sr && y == yr);
  }
  CHECK(lk_dispose(c) == LK_OK);
  std::vector<lk_log_entry> log(1024);
  uint32_t cnt = 0;
  CHECK(lk_read_log(c, 0, log.data(), 1024, &cnt) == LK_OK && cnt == 1000);
  for (uint32_t i = 0; i < cnt; ++i) CHECK(log[i].seq == i + 1);
  lk_free(c);
  printf("OK %s\n", g_case);
}

// Several clusters driven concurrently, depth 4, every result exact, exactly once, FIFO.
static void concurrent_clusters() {
  g_case = "concurrent_clusters";
  const uint32_t W = 8, items = 400, depth = 4;
  lk_ctx *c = open_ctx(W, depth, LK_CLUSTERS_PER_WORKER, 20000, 512);
  std::atomic<int> bad{0};
  std::vector<std::thread> th;
  for (uint32_t w = 0; w < W; ++w) {
    th.emplace_back([&, w] {
      const uint64_t n = 100 + w;
      std::vector<std::vector<int32_t>> xs(items, std::vector<int32_t>(n)), ys(items, std::vector<int32_t>(n));
      std::mt19937 rng(100 + w);
      for (auto &x : xs)
        for (auto &v : x) v = static_cast<int32_t>(rng());
      std::vector<uint64_t> tick(items);
      std::vector<int64_t> res(items);
      uint32_t posted = 0, done = 0;
      while (done < items) {
        while (posted < items && posted - done < depth) {
          lk_desc d = desc(LK_OP_AFFINE_SUM_I32, n, static_cast<int32_t>(posted) + 3, -7);
          const int rc = lk_submit(c, w, &d, xs[posted].data(), ys[posted].data(), &tick[posted]);
          if (rc == LK_EAGAIN) break;
          if (rc != LK_OK) bad.fetch_add(1);
          ++posted;
        }
        if (lk_wait(c, w, tick[done], 5000000000ll, &res[done]) != LK_OK) bad.fetch_add(1);
        ++done;
      }
      std::vector<int32_t> yr(n);
      for (uint32_t i = 0; i < items; ++i) {
        int64_t sr;
        affine_ref(xs[i].data(), n, static_cast<int32_t>(i) + 3, -7, yr.data(), &sr);
        if (sr != res[i] || yr != ys[i] || tick[i] != i + 1) bad.fetch_add(1);
      }
    });
  }
  for (auto &t : th) t.join();
  CHECK(bad.load() == 0);
  CHECK(lk_dispose(c) == LK_OK);
  std::vector<lk_log_entry> log(512);
  for (uint32_t w = 0; w < W; ++w) {
    uint32_t cnt = 0;
    CHECK(lk_read_log(c, w, log.data(), 512, &cnt) == LK_OK && cnt == items);
    for (uint32_t i = 0; i < cnt; ++i) CHECK(log[i].seq == i + 1);
  }
  lk_free(c);
  printf("OK %s\n", g_case);
}

// Errors forced from the host: EAGAIN, EINVAL, ETIMEDOUT on a frozen worker, ESTATE.
static void error_paths() {
  g_case = "error_paths";
  lk_ctx *c = open_ctx(2, 1, LK_CLUSTERS_PER_WORKER);
  std::vector<int32_t> x(64, 1), y(64);
  uint64_t t;
  lk_desc bad = desc(99, 1);
  CHECK(lk_submit(c, 0, &bad, x.data(), y.data(), &t) == LK_EINVAL);
  lk_desc d = desc(LK_OP_AFFINE_SUM_I32, 16);
  CHECK(lk_submit(c, 7, &d, x.data(), y.data(), &t) == LK_EINVAL);                            // no cluster 7
  CHECK(lk_submit(c, 0, &d, reinterpret_cast<char *>(x.data()) + 2, y.data(), &t) == LK_EINVAL);  // misaligned
  // a hung worker: the wait times out, and succeeds once the worker runs again
  lkfake_freeze(0);
  lk_desc nop = desc(LK_OP_NOP, 0);
  uint64_t t0;
  CHECK(lk_submit(c, 0, &nop, nullptr, nullptr, &t0) == LK_OK);
  CHECK(lk_submit(c, 0, &nop, nullptr, nullptr, &t) == LK_EAGAIN);  // depth 1: ring full
  CHECK(lk_wait(c, 0, t0, 20000000ll, nullptr) == LK_ETIMEDOUT);
  int done = 1;
  CHECK(lk_poll(c, 0, t0, &done) == LK_OK && done == 0);
  lk_completion ci;
  CHECK(lk_try_wait(c, 0, t0, &ci) == LK_EAGAIN);  // not finished: the ticket stays valid
  lkfake_freeze(-1);
  int rc;
  while ((rc = lk_try_wait(c, 0, t0, &ci)) == LK_EAGAIN) std::this_thread::yield();
  CHECK(rc == LK_OK && ci.result == 0);
  CHECK(lk_try_wait(c, 0, t0, &ci) == LK_EINVAL);  // released
  CHECK(lk_submit(c, 0, &nop, nullptr, nullptr, &t0) == LK_OK);
  lkfake_freeze(-1);
  CHECK(lk_wait(c, 0, t0, 5000000000ll, nullptr) == LK_OK);
  CHECK(lk_wait(c, 0, t0, 0, nullptr) == LK_EINVAL);  // already released
  CHECK(lk_wait(c, 1, 5, 0, nullptr) == LK_EINVAL);   // never posted
  CHECK(lk_dispose(c) == LK_OK);
  CHECK(lk_dispose(c) == LK_OK);  // idempotent
  CHECK(lk_submit(c, 0, &nop, nullptr, nullptr, &t) == LK_ESTATE);
  CHECK(lk_wait(c, 0, 1, 0, nullptr) == LK_ESTATE);
  lk_free(c);
  printf("OK %s\n", g_case);
}

// Pinned input: a flagged item whose x matches the worker's pinned copy computes with that
// copy (so a change to x in memory goes unseen until PIN_RELOAD), unflagged items read
// memory and leave the copy in place, and lk_submit rejects shapes the buffer cannot take.
static void pinned_input() {
  g_case = "pinned_input";
  lk_ctx *c = open_ctx(2, 1, LK_CLUSTERS_PER_WORKER);
  lk_info info{};
  CHECK(lk_get_info(c, &info) == LK_OK && info.pin_capacity >= 64 * 1024);
  const uint64_t n = 4096;
  alignas(64) static float x[8192], x2[8192], y[8192], yr[8192];
  std::mt19937 rng(11);
  std::uniform_real_distribution<float> u(-1.f, 1.f);
  for (uint64_t i = 0; i < 8192; ++i) x[i] = u(rng), x2[i] = u(rng), y[i] = u(rng);
  memcpy(yr, y, sizeof y);
  auto run = [&](lk_desc d, const float *xp) {
    uint64_t t;
    CHECK(lk_submit(c, 0, &d, xp, y, &t) == LK_OK);
    CHECK(lk_wait(c, 0, t, 5000000000ll, nullptr) == LK_OK);
  };
  auto ref = [&](float alpha, const float *xs) {
    for (uint64_t i = 0; i < n; ++i) yr[i] = std::fmaf(alpha, xs[i], yr[i]);
  };
  lk_desc d = desc(LK_OP_SAXPY_F32, n, 0, 0, 0.5f);
  d.flags = LK_DF_PIN_INPUT;
  run(d, x);  // first flagged item: loads and pins x
  ref(0.5f, x);
  float old[4096];
  memcpy(old, x, sizeof old);
  for (uint64_t i = 0; i < n; ++i) x[i] += 1.f;  // broken promise: the pinned copy is used
  run(d, x);
  ref(0.5f, old);
  CHECK(memcmp(y, yr, n * 4) == 0);
  lk_desc plain = desc(LK_OP_SAXPY_F32, n, 0, 0, -1.25f);
  run(plain, x);  // unflagged: memory
  ref(-1.25f, x);
  run(d, x);  // the copy is still the old x
  ref(0.5f, old);
  CHECK(memcmp(y, yr, n * 4) == 0);
  lk_desc rl = d;
  rl.flags = LK_DF_PIN_RELOAD;
  run(rl, x);
  ref(0.5f, x);
  run(d, x);
  ref(0.5f, x);
  run(d, x2);  // another address: loads and replaces
  ref(0.5f, x2);
  CHECK(memcmp(y, yr, n * 4) == 0);
  // AXPY with a pinned x
  alignas(64) static float yy[4096], out[4096];
  for (uint64_t i = 0; i < n; ++i) yy[i] = u(rng);
  lk_desc ax = desc(LK_OP_AXPY_F32, n, 0, 0, 3.f, reinterpret_cast<uint64_t>(yy));
  ax.flags = LK_DF_PIN_INPUT;
  uint64_t t;
  CHECK(lk_submit(c, 1, &ax, x2, out, &t) == LK_OK && lk_wait(c, 1, t, 5000000000ll, nullptr) == LK_OK);
  for (uint64_t i = 0; i < n; ++i) CHECK(out[i] == std::fmaf(3.f, x2[i], yy[i]));
  // Several slices per worker: worker 0 holds x and x2 already; two more make four, each
  // served from its copy after x changes in memory; a fifth address resets the table,
  // after which an earlier one is loaded again from memory.
  {
    alignas(64) static float xs[3][4096], old0[4096], old1[4096], old2[4096];
    for (auto &row : xs)
      for (float &v : row) v = u(rng);
    run(d, xs[0]);
    ref(0.5f, xs[0]);
    run(d, xs[1]);
    ref(0.5f, xs[1]);
    memcpy(old0, xs[0], sizeof old0);
    memcpy(old1, xs[1], sizeof old1);
    memcpy(old2, x2, sizeof old2);
    for (uint64_t i = 0; i < n; ++i) xs[0][i] -= 2.f, xs[1][i] *= 3.f, x2[i] += 7.f;
    run(d, xs[1]);
    ref(0.5f, old1);
    run(d, x2);
    ref(0.5f, old2);
    run(d, xs[0]);
    ref(0.5f, old0);
    CHECK(memcmp(y, yr, n * 4) == 0);
    run(d, xs[2]);  // fifth slice: the table is reset
    ref(0.5f, xs[2]);
    run(d, xs[0]);  // loaded again: the changed x
    ref(0.5f, xs[0]);
    run(d, xs[2]);  // still pinned beside it
    ref(0.5f, xs[2]);
    CHECK(memcmp(y, yr, n * 4) == 0);
  }
  // The integer ops: the pinned words stand in for x in the sum and in AFFINE's y.
  alignas(64) static int32_t xi[4096], yi[4096];
  for (uint64_t i = 0; i < n; ++i) xi[i] = static_cast<int32_t>(rng());
  auto isum = [&](int32_t a, int32_t b, const int32_t *xs, bool affine) {
    int64_t s = 0;
    for (uint64_t i = 0; i < n; ++i) {
      const int32_t v = affine ? static_cast<int32_t>(static_cast<uint32_t>(a) * static_cast<uint32_t>(xs[i]) +
                                                      static_cast<uint32_t>(b))
                               : xs[i];
      s += v;
      if (affine) CHECK(yi[i] == v);
    }
    return s;
  };
  auto irun = [&](lk_desc di, const int32_t *xp) {
    int64_t r = 0;
    CHECK(lk_submit(c, 1, &di, xp, di.op == LK_OP_SUM_I32_I64 ? nullptr : yi, &t) == LK_OK);
    CHECK(lk_wait(c, 1, t, 5000000000ll, &r) == LK_OK);
    return r;
  };
  lk_desc af = desc(LK_OP_AFFINE_SUM_I32, n, -7, 13);
  af.flags = LK_DF_PIN_INPUT;
  CHECK(irun(af, xi) == isum(-7, 13, xi, true));  // loads and pins xi (replacing x2)
  int32_t iold[4096];
  memcpy(iold, xi, sizeof iold);
  for (uint64_t i = 0; i < n; ++i) xi[i] ^= 0x5a5a;
  CHECK(irun(af, xi) == isum(-7, 13, iold, true));  // the pinned copy
  lk_desc su = desc(LK_OP_SUM_I32_I64, n);
  su.flags = LK_DF_PIN_INPUT;
  CHECK(irun(su, xi) == isum(0, 0, iold, false));  // same address and length: the copy again
  su.flags = LK_DF_PIN_RELOAD;
  CHECK(irun(su, xi) == isum(0, 0, xi, false));
  CHECK(irun(af, xi) == isum(-7, 13, xi, true));
  // shapes the pinned path refuses
  lk_desc e = d;
  e.flags = 0x4;
  CHECK(lk_submit(c, 0, &e, x, y, &t) == LK_EINVAL);
  e = desc(LK_OP_COPY_F32, 64);
  e.flags = LK_DF_PIN_INPUT;
  CHECK(lk_submit(c, 0, &e, x, y, &t) == LK_EINVAL);
  e = desc(LK_OP_SUM_I32_I64, 64);
  e.flags = LK_DF_PIN_INPUT;
  CHECK(lk_submit(c, 0, &e, xi, reinterpret_cast<int32_t *>(yi) + 1, &t) == LK_OK);  // SUM ignores out
  CHECK(lk_wait(c, 0, t, 5000000000ll, nullptr) == LK_OK);
  e = desc(LK_OP_AFFINE_SUM_I32, 64);
  e.flags = LK_DF_PIN_INPUT;
  CHECK(lk_submit(c, 0, &e, xi, yi + 1, &t) == LK_EINVAL);  // AFFINE's out must be aligned
  e = d;
  CHECK(lk_submit(c, 0, &e, x + 1, y + 1, &t) == LK_EINVAL);  // 4- but not 16-byte aligned
  e.n = n - 2;
  CHECK(lk_submit(c, 0, &e, x, y, &t) == LK_EINVAL);  // not a multiple of 4
  e.n = info.pin_capacity / 4 + 4;
  std::vector<float> big(e.n + 64);
  float *bp = reinterpret_cast<float *>((reinterpret_cast<uintptr_t>(big.data()) + 15) & ~uintptr_t(15));
  CHECK(lk_submit(c, 0, &e, bp, bp, &t) == LK_EINVAL);  // larger than the LDS buffer
  e.n = 0;
  CHECK(lk_submit(c, 0, &e, nullptr, nullptr, &t) == LK_OK && lk_wait(c, 0, t, 5000000000ll, nullptr) == LK_OK);
  uint64_t in_a = reinterpret_cast<uint64_t>(x), out_a = reinterpret_cast<uint64_t>(y);
  lk_tile tiles[4];
  uint32_t item_of[4], nt = 0;
  CHECK(lk_batch_plan(&d, &in_a, &out_a, 1, 4096, tiles, item_of, 4, &nt) == LK_EINVAL);
  CHECK(lk_dispose(c) == LK_OK);
  lk_free(c);
  printf("OK %s\n", g_case);
}

// One item sliced over a cluster of every worker: exact sum, output and per-member partials.
static void cluster_split() {
  g_case = "cluster_split";
  lk_ctx *c = open_ctx(8, 1, LK_CLUSTERS_ONE);
  const uint64_t n = 100003;
  std::vector<int32_t> x(n), y(n), yr(n);
  std::mt19937 rng(7);
  for (auto &v : x) v = static_cast<int32_t>(rng());
  std::vector<int64_t> parts(8, -1);
  lk_desc d = desc(LK_OP_AFFINE_SUM_I32, n, -5, 11, 0.f, reinterpret_cast<uint64_t>(parts.data()));
  uint64_t t;
  int64_t s = 0, sr = 0;
  CHECK(lk_submit(c, 0, &d, x.data(), y.data(), &t) == LK_OK);
  CHECK(lk_wait(c, 0, t, 5000000000ll, &s) == LK_OK);
  affine_ref(x.data(), n, -5, 11, yr.data(), &sr);
  CHECK(s == sr && y == yr);
  // the same item released through the non-blocking form, with one member held back:
  // nothing is released until all 8 have finished
  std::fill(y.begin(), y.end(), 0);
  lkfake_freeze(5);
  CHECK(lk_submit(c, 0, &d, x.data(), y.data(), &t) == LK_OK);
  lk_completion ci;
  std::this_thread::sleep_for(std::chrono::milliseconds(20));
  CHECK(lk_try_wait(c, 0, t, &ci) == LK_EAGAIN);
  lkfake_freeze(-1);
  int rc;
  while ((rc = lk_try_wait(c, 0, t, &ci)) == LK_EAGAIN) std::this_thread::yield();
  CHECK(rc == LK_OK && ci.result == sr && y == yr && ci.t_pick_min <= ci.t_done_max);
  int64_t psum = 0;
  for (int64_t v : parts) psum += v;
  CHECK(psum == sr);
  CHECK(lk_dispose(c) == LK_OK);
  lk_free(c);
  printf("OK %s\n", g_case);
}

// A batch of uneven items cut into tiles and claimed by every worker of one cluster.
static void batch_tiles() {
  g_case = "batch_tiles";
  lk_ctx *c = open_ctx(8, 2, LK_CLUSTERS_ONE);
  const uint32_t items = 40;
  std::mt19937 rng(9);
  std::vector<std::vector<int32_t>> xs(items), ys(items);
  std::vector<lk_desc> ds(items);
  std::vector<uint64_t> ia(items), oa(items);
  for (uint32_t i = 0; i < items; ++i) {
    const uint64_t n = 1 + rng() % 5000;
    xs[i].resize(n);
    ys[i].assign(n, 0);
    for (auto &v : xs[i]) v = static_cast<int32_t>(rng());
    ds[i] = desc(LK_OP_AFFINE_SUM_I32, n, static_cast<int32_t>(i), 1);
    ia[i] = reinterpret_cast<uint64_t>(xs[i].data());
    oa[i] = reinterpret_cast<uint64_t>(ys[i].data());
  }
  uint32_t nt = 0;
  CHECK(lk_batch_plan(ds.data(), ia.data(), oa.data(), items, 1024, nullptr, nullptr, 0, &nt) == LK_EINVAL && nt > 0);
  std::vector<lk_tile> tiles(nt);
  std::vector<uint32_t> owner(nt);
  CHECK(lk_batch_plan(ds.data(), ia.data(), oa.data(), items, 1024, tiles.data(), owner.data(), nt, &nt) == LK_OK);
  for (int rep = 0; rep < 3; ++rep) {  // the slot counters keep advancing across batches
    std::vector<int64_t> parts(nt, 0);
    uint64_t t;
    int64_t executed = 0;
    CHECK(lk_submit_batch(c, 0, tiles.data(), nt, parts.data(), &t) == LK_OK);
    CHECK(lk_wait(c, 0, t, 5000000000ll, &executed) == LK_OK && executed == nt);
    std::vector<int64_t> sum(items, 0);
    for (uint32_t k = 0; k < nt; ++k) sum[owner[k]] += parts[k];
    for (uint32_t i = 0; i < items; ++i) {
      std::vector<int32_t> yr(xs[i].size());
      int64_t sr;
      affine_ref(xs[i].data(), xs[i].size(), static_cast<int32_t>(i), 1, yr.data(), &sr);
      CHECK(sum[i] == sr && ys[i] == yr);
    }
  }
  CHECK(lk_dispose(c) == LK_OK);
  lk_free(c);
  printf("OK %s\n", g_case);
}

// Serving: Poisson-like arrivals on 8 fake workers, 4 scheduler threads, retained outputs.
static void serving() {
  g_case = "serving";
  lk_ctx *c = open_ctx(8, 4, LK_CLUSTERS_PER_WORKER);
  const uint32_t count = 300;
  std::mt19937 rng(11);
  std::vector<std::vector<int32_t>> xs(count);
  std::vector<std::vector<float>> xf(count), yf(count);
  std::vector<lks_request> req(count);
  double t_us = 0;
  uint64_t total_out = 0;
  for (uint32_t i = 0; i < count; ++i) {
    lks_request &r = req[i];
    memset(&r, 0, sizeof r);
    t_us += (rng() % 200) * 0.5;
    r.arrival_us = t_us;
    const uint32_t kind = rng() % 3;
    r.n = 1 + rng() % 20000;
    xs[i].resize(r.n);
    for (auto &v : xs[i]) v = static_cast<int32_t>(rng());
    r.a = static_cast<int32_t>(rng());
    r.b = static_cast<int32_t>(rng());
    if (kind == 0) {
      r.op = LK_OP_AFFINE_SUM_I32;
      r.in = reinterpret_cast<uint64_t>(xs[i].data());
    } else if (kind == 1) {
      r.op = LK_OP_SUM_I32_I64;
      r.in = reinterpret_cast<uint64_t>(xs[i].data());
    } else {
      r.op = LK_OP_AXPY_F32;
      xf[i].resize(r.n);
      yf[i].resize(r.n);
      for (uint64_t k = 0; k < r.n; ++k) {
        xf[i][k] = static_cast<float>(static_cast<int32_t>(rng())) * 1e-9f;
        yf[i][k] = static_cast<float>(static_cast<int32_t>(rng())) * 1e-9f;
      }
      r.alpha = 0.75f;
      r.in = reinterpret_cast<uint64_t>(xf[i].data());
      r.in2 = reinterpret_cast<uint64_t>(yf[i].data());
    }
    total_out += (r.n * 4 + 255) / 256 * 256;
  }
  const uint64_t arena_bytes = (total_out + (1u << 20)) * 4;  // every shard holds all of its outputs
  void *arena = aligned_alloc(256, arena_bytes);
  CHECK(arena != nullptr);
  lks_config cfg;
  memset(&cfg, 0, sizeof cfg);
  cfg.arena = reinterpret_cast<uint64_t>(arena);
  cfg.arena_bytes = arena_bytes;
  cfg.tile_elems = 4096;
  cfg.threads = 4;
  cfg.retain = 1;
  cfg.timeout_ns = 5000000000ll;
  std::vector<lks_outcome> out(count);
  lks_stats st;
  // Rejected configurations and traces name their reason in lk_last_error.
  {
    lks_config bad = cfg;
    bad.threads = 9;  // more schedulers than the 8 workers
    CHECK(lks_run(c, &bad, req.data(), count, out.data(), &st) == LK_EINVAL);
    CHECK(strstr(lk_last_error(), "scheduler threads") != nullptr);
    bad = cfg;
    bad.tile_elems = 1000;
    CHECK(lks_run(c, &bad, req.data(), count, out.data(), &st) == LK_EINVAL);
    CHECK(strstr(lk_last_error(), "tile_elems") != nullptr);
    std::vector<lks_request> late(req.begin(), req.begin() + 3);
    late[2].arrival_us = late[1].arrival_us - 1.0;
    CHECK(lks_run(c, &cfg, late.data(), 3, out.data(), &st) == LK_EINVAL);
    CHECK(strstr(lk_last_error(), "request 2 arrives before") != nullptr);
  }
  CHECK(lks_run(c, &cfg, req.data(), count, out.data(), &st) == LK_OK);
  uint64_t tiles = 0;
  for (uint32_t i = 0; i < count; ++i) {
    const lks_request &r = req[i];
    CHECK(out[i].status == LK_OK && out[i].done_us >= out[i].admit_us);
    tiles += out[i].tiles;
    if (r.op == LK_OP_AFFINE_SUM_I32) {
      std::vector<int32_t> yr(r.n);
      int64_t sr;
      affine_ref(xs[i].data(), r.n, r.a, r.b, yr.data(), &sr);
      CHECK(out[i].result == sr && memcmp(reinterpret_cast<void *>(out[i].out), yr.data(), r.n * 4) == 0);
    } else if (r.op == LK_OP_SUM_I32_I64) {
      int64_t sr = 0;
      for (int32_t v : xs[i]) sr += v;
      CHECK(out[i].result == sr);
    } else {
      const float *o = reinterpret_cast<const float *>(out[i].out);
      for (uint64_t k = 0; k < r.n; ++k) CHECK(o[k] == std::fmaf(r.alpha, xf[i][k], yf[i][k]));
    }
  }
  CHECK(st.tiles == tiles);
  CHECK(lk_dispose(c) == LK_OK);
  lk_free(c);
  free(arena);
  printf("OK %s\n", g_case);
}

// Serving stopped by an error: one worker hangs, its scheduler times out, every scheduler
// stops, and lks_run returns only once the tiles already posted have finished (the hung
// worker is released 600 ms in, after the 200 ms timeout has fired): posted = taken +
// drained, and the context is still running and usable afterwards.
static void serving_error_drains() {
  g_case = "serving_error_drains";
  lk_ctx *c = open_ctx(8, 4, LK_CLUSTERS_PER_WORKER);
  const uint32_t count = 64;
  const uint64_t n = 20000;
  std::vector<std::vector<int32_t>> xs(count, std::vector<int32_t>(n));
  std::vector<lks_request> req(count);
  for (uint32_t i = 0; i < count; ++i) {
    for (uint64_t k = 0; k < n; ++k) xs[i][k] = static_cast<int32_t>(k * 2654435761u + i);
    memset(&req[i], 0, sizeof req[i]);
    req[i].arrival_us = 0.0;
    req[i].op = LK_OP_SUM_I32_I64;
    req[i].n = n;
    req[i].in = reinterpret_cast<uint64_t>(xs[i].data());
  }
  lks_config cfg;
  memset(&cfg, 0, sizeof cfg);
  cfg.tile_elems = 4096;
  cfg.threads = 4;
  cfg.timeout_ns = 200000000ll;
  std::vector<lks_outcome> out(count);
  lks_stats st;
  std::atomic<bool> released{false};
  lkfake_freeze(3);
  std::thread unfreeze([&] {
    std::this_thread::sleep_for(std::chrono::milliseconds(600));
    released.store(true);
    lkfake_freeze(-1);
  });
  const int rc = lks_run(c, &cfg, req.data(), count, out.data(), &st);
  const bool after_release = released.load();
  unfreeze.join();
  CHECK(rc == LK_ETIMEDOUT);
  CHECK(after_release);
  CHECK(st.posted > 0 && st.drained > 0 && st.posted == st.tiles + st.drained);
  for (uint32_t i = 0; i < count; ++i) {
    if (out[i].status != LK_OK) continue;
    int64_t sr = 0;
    for (int32_t v : xs[i]) sr += v;
    CHECK(out[i].result == sr);
  }
  lk_info info;
  CHECK(lk_get_info(c, &info) == LK_OK && info.state == 0);
  for (uint32_t cl = 0; cl < 8; ++cl) {
    lk_desc nop = desc(LK_OP_NOP, 0);
    uint64_t t;
    CHECK(lk_submit(c, cl, &nop, nullptr, nullptr, &t) == LK_OK);
    CHECK(lk_wait(c, cl, t, 5000000000ll, nullptr) == LK_OK);
  }
  CHECK(lk_dispose(c) == LK_OK);
  lk_free(c);
  printf("OK %s\n", g_case);
}

// Idle watchdog: workers leave after the idle timeout; later calls see ESTATE.
static void idle_watchdog() {
  g_case = "idle_watchdog";
  lk_ctx *c = open_ctx(4, 1, LK_CLUSTERS_PER_WORKER, 100);
  std::this_thread::sleep_for(std::chrono::milliseconds(400));
  lk_info info;
  CHECK(lk_get_info(c, &info) == LK_OK && info.workers_exited == 4);
  lk_desc nop = desc(LK_OP_NOP, 0);
  uint64_t t;
  CHECK(lk_submit(c, 0, &nop, nullptr, nullptr, &t) == LK_ESTATE);
  CHECK(lk_dispose(c) == LK_OK);
  lk_free(c);
  printf("OK %s\n", g_case);
}

// Dispose with items still in flight drains them first.
static void dispose_in_flight() {
  g_case = "dispose_in_flight";
  lk_ctx *c = open_ctx(2, 4, LK_CLUSTERS_PER_WORKER);
  std::vector<int32_t> x(50000, 3), y(50000);
  lk_desc d = desc(LK_OP_AFFINE_SUM_I32, 50000, 2, 1);
  uint64_t t;
  for (int i = 0; i < 4; ++i) CHECK(lk_submit(c, 0, &d, x.data(), y.data(), &t) == LK_OK);
  CHECK(lk_dispose(c) == LK_OK);
  for (int32_t v : y) CHECK(v == 7);
  lk_info info;
  CHECK(lk_get_info(c, &info) == LK_OK && info.state == 1 && info.workers_exited == 2);
  lk_free(c);
  printf("OK %s\n", g_case);
}

// Dispose while a worker is hung: LK_ETIMEDOUT and a poisoned context whose resources stay
// allocated; once the worker runs again a second dispose completes.
static void dispose_hung_worker() {
  g_case = "dispose_hung_worker";
  lk_ctx *c = open_ctx(2, 1, LK_CLUSTERS_PER_WORKER, 100);  // dispose gives up after 5 s + 0.1 s
  lkfake_freeze(1);
  CHECK(lk_dispose(c) == LK_ETIMEDOUT);
  lk_info info;
  CHECK(lk_get_info(c, &info) == LK_OK && info.state == 2);
  lk_desc nop = desc(LK_OP_NOP, 0);
  uint64_t t;
  CHECK(lk_submit(c, 0, &nop, nullptr, nullptr, &t) == LK_ESTATE);
  lkfake_freeze(-1);
  CHECK(lk_dispose(c) == LK_OK);
  CHECK(lk_get_info(c, &info) == LK_OK && info.state == 1);
  lk_free(c);
  printf("OK %s\n", g_case);
}

// A second context that would need more CUs than are left is refused at once.
static void cu_reservation() {
  g_case = "cu_reservation";
  lk_ctx *a = open_ctx(12, 1, LK_CLUSTERS_PER_WORKER);
  lk_config cfg;
  lk_config_default(&cfg);
  cfg.n_workers = 8;  // 12 + 8 > 16 fake CUs
  lk_ctx *b = nullptr;
  CHECK(lk_init(&cfg, &b) == LK_ENODEV && b == nullptr);
  cfg.n_workers = 4;
  CHECK(lk_init(&cfg, &b) == LK_OK);
  CHECK(lk_dispose(b) == LK_OK && lk_dispose(a) == LK_OK);
  lk_free(b);
  lk_free(a);
  printf("OK %s\n", g_case);
}

// Workers restricted to XCDs 0 and 2 (2 fake CUs each): 4 workers, all on those XCDs,
// two XCD clusters computing exactly; the masked context holds every CU; masks beyond
// the device and worker counts beyond the masked CUs are refused.
static void xcd_mask() {
  g_case = "xcd_mask";
  lk_config cfg;
  lk_config_default(&cfg);
  cfg.xcd_mask = 0x5;
  cfg.cluster_policy = LK_CLUSTERS_PER_XCD;
  cfg.idle_timeout_ms = 20000;
  lk_ctx *c = nullptr;
  CHECK(lk_init(&cfg, &c) == LK_OK && c);
  lk_info info{};
  CHECK(lk_get_info(c, &info) == LK_OK);
  CHECK(info.n_workers == 4 && info.n_clusters == 2 && info.xcd_mask == 0x5 && info.xcd_count == 2);
  for (uint32_t w = 0; w < 4; ++w) {
    uint32_t xcc = 9, se, sh, cu;
    CHECK(lk_topology(c, w, &xcc, &se, &sh, &cu) == LK_OK && (xcc == 0 || xcc == 2));
  }
  const uint64_t n = 5000;
  std::vector<int32_t> x(n), y(n), yr(n);
  for (uint64_t i = 0; i < n; ++i) x[i] = static_cast<int32_t>(i * 2654435761u);
  for (uint32_t cl = 0; cl < 2; ++cl) {
    lk_desc d = desc(LK_OP_AFFINE_SUM_I32, n, 3 + cl, -7);
    uint64_t t;
    int64_t s = 0, sr = 0;
    CHECK(lk_submit(c, cl, &d, x.data(), y.data(), &t) == LK_OK);
    CHECK(lk_wait(c, cl, t, 5000000000ll, &s) == LK_OK);
    affine_ref(x.data(), n, 3 + cl, -7, yr.data(), &sr);
    CHECK(s == sr && y == yr);
  }
  lk_config other;
  lk_config_default(&other);
  other.n_workers = 1;
  lk_ctx *b = nullptr;
  CHECK(lk_init(&other, &b) == LK_ENODEV && b == nullptr);  // the masked context holds every CU
  CHECK(lk_dispose(c) == LK_OK);
  lk_free(c);
  cfg.xcd_mask = 0x100;  // 8 fake XCDs
  CHECK(lk_init(&cfg, &c) == LK_EINVAL);
  cfg.xcd_mask = 0x1;
  cfg.n_workers = 3;  // XCD 0 has 2 CUs
  CHECK(lk_init(&cfg, &c) == LK_EINVAL);
  printf("OK %s\n", g_case);
}

int main() {
  single_worker_1000();
  concurrent_clusters();
  error_paths();
  pinned_input();
  cluster_split();
  batch_tiles();
  serving();
  serving_error_drains();
  idle_watchdog();
  dispose_in_flight();
  dispose_hung_worker();
  cu_reservation();
  xcd_mask();
  printf("ALL OK\n");
  return 0;
}
