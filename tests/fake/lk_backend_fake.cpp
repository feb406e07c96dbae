// Fake device for host-logic tests: implements the host library's backend (lk_backend.h)
// with ordinary memory and one std::thread per worker, speaking the same mailbox
// protocol as the gfx950 worker (boot claim and INIT, tagged command slots, status
// records published last-word-release, EXIT, idle watchdog).  Test infrastructure only:
// it is linked into the test binary built by tests/test_fake_device.py, never into
// liblk.so.  Hooks: lkfake_freeze(mailbox) stops one worker from polling (a hung worker),
// lkfake_freeze(-1) releases it.
#include <immintrin.h>
#include <stdint.h>

#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "lk.h"
#include "lk_backend.h"
#include "lk_common.h"
#include "lk_wire.h"

namespace {

using clk = std::chrono::steady_clock;
std::atomic<int> g_frozen{-1};
const auto g_t0 = clk::now();

uint64_t wall_ticks() {  // 100 MHz, like the device wall clock
  return static_cast<uint64_t>(std::chrono::duration_cast<std::chrono::nanoseconds>(clk::now() - g_t0).count() / 10);
}
uint64_t ld_acq(const uint64_t *p) { return __atomic_load_n(p, __ATOMIC_ACQUIRE); }
void st_rel(uint64_t *p, uint64_t v) { __atomic_store_n(p, v, __ATOMIC_RELEASE); }
void st_rlx(uint64_t *p, uint64_t v) { __atomic_store_n(p, v, __ATOMIC_RELAXED); }

void relax(uint32_t &spins) {
  if ((++spins & 255u) == 0) std::this_thread::yield();
  else _mm_pause();
}

struct Slice {
  uint32_t op;
  uint64_t n;
  uint64_t in, out, in2;
  uint32_t a, b;
};

int64_t run_slice(const Slice &s) {
  int64_t acc = 0;
  auto *xi = reinterpret_cast<const int32_t *>(s.in);
  switch (s.op) {
    case 1: {  // AFFINE_SUM_I32
      auto *y = reinterpret_cast<int32_t *>(s.out);
      for (uint64_t i = 0; i < s.n; ++i) {
        const int32_t v = static_cast<int32_t>(s.a * static_cast<uint32_t>(xi[i]) + s.b);
        y[i] = v;
        acc += v;
      }
      break;
    }
    case 2:  // SUM_I32_I64
      for (uint64_t i = 0; i < s.n; ++i) acc += xi[i];
      break;
    case 3: {  // SAXPY_F32 in place
      float alpha;
      memcpy(&alpha, &s.b, 4);
      auto *x = reinterpret_cast<const float *>(s.in);
      auto *y = reinterpret_cast<float *>(s.out);
      for (uint64_t i = 0; i < s.n; ++i) y[i] = std::fmaf(alpha, x[i], y[i]);
      break;
    }
    case 4: {  // COPY_F32
      memcpy(reinterpret_cast<void *>(s.out), reinterpret_cast<const void *>(s.in), s.n * 4);
      break;
    }
    case 5: {  // SPIN: a iterations of busy work
      volatile uint32_t v = 1;
      for (uint32_t i = 0; i < s.a; ++i) v = v * 1664525u + 1013904223u;
      break;
    }
    case 7: {  // AXPY_F32 out of place
      float alpha;
      memcpy(&alpha, &s.b, 4);
      auto *x = reinterpret_cast<const float *>(s.in);
      auto *y = reinterpret_cast<const float *>(s.in2);
      auto *o = reinterpret_cast<float *>(s.out);
      for (uint64_t i = 0; i < s.n; ++i) o[i] = std::fmaf(alpha, x[i], y[i]);
      break;
    }
    default:
      break;
  }
  return acc;
}

void worker(lkw_params p, uint32_t wg, std::atomic<uint32_t> *running) {
  // Distinct fake placement per workgroup: XCC = wg % 8, CU/SH/SE from the rest.
  const uint32_t xcc = wg % 8, cu = (wg / 8) % 16, sh = (wg / 128) % 2, se = (wg / 256) % 4;
  const uint32_t m = ((p.xcc_mask >> xcc) & 1u) ? __atomic_fetch_add(p.claim, 1u, __ATOMIC_RELAXED) : ~0u;
  if (m >= p.n_workers) {
    running->fetch_sub(1, std::memory_order_release);
    return;
  }
  const uint32_t hw = (cu << 8) | (sh << 12) | (se << 13);
  lkw_worker *wr = p.workers + m;
  __atomic_store_n(&wr->hwid, hw, __ATOMIC_RELAXED);
  __atomic_store_n(&wr->xcc, xcc, __ATOMIC_RELAXED);
  __atomic_store_n(&wr->wg, wg, __ATOMIC_RELAXED);
  __atomic_store_n(&wr->t_boot, wall_ticks(), __ATOMIC_RELAXED);
  st_rel(&wr->word, LKW_WORD(0, LKW_FROM_INIT));

  const uint64_t stride = LKW_RING_STRIDE(p.depth);
  lkw_cmd *ring = p.cmd + m * stride;
  lkw_status *sring = p.status + m * stride;
  uint64_t seq = 0;
  // Model of the pinned input: up to LKW_PIN_SLOTS copies of x's 32-bit words per worker,
  // placed one after another in an LDS of p.lds_bytes; a slice that does not fit after
  // the others (or finds every slot taken) replaces all of them.
  std::vector<uint32_t> lds(p.lds_bytes / 4);
  struct PinSlot {
    uint64_t addr = 0, n = 0, off = 0;  // off in 32-bit words
  };
  std::vector<PinSlot> pins;
  for (;;) {
    const uint64_t want = seq + 1;
    const uint32_t slot = static_cast<uint32_t>(want % p.depth);
    const uint64_t *src = ring[slot].w;
    const uint64_t t0 = wall_ticks();
    uint64_t w[LKW_CMD_WORDS];
    uint32_t spins = 0;
    bool timed_out = false;
    for (;;) {
      if (g_frozen.load(std::memory_order_relaxed) == static_cast<int>(m)) {  // hung: no poll, no watchdog
        relax(spins);
        continue;
      }
      w[0] = ld_acq(src);
      bool ok = LKW_SEQ(w[0]) == want;
      for (int i = 1; ok && i < LKW_CMD_WORDS; ++i) {
        w[i] = ld_acq(src + i);
        ok = (w[i] >> LKW_TAG_SHIFT) == (want & 0xffffu);
      }
      if (ok) break;
      if (wall_ticks() - t0 > p.idle_ticks) {
        timed_out = true;
        break;
      }
      relax(spins);
    }
    const uint64_t t_pick = wall_ticks();
    if (timed_out) {
      __atomic_store_n(&wr->t_exit, t_pick, __ATOMIC_RELAXED);
      st_rel(&wr->word, LKW_WORD(seq, LKW_FROM_TIMEDOUT));
      break;
    }
    const uint32_t code = LKW_CODE(w[0]);
    uint32_t reply = LKW_FROM_FINISHED;
    int64_t partial = 0;
    Slice s{};
    s.n = w[LKW_W_N] & LKW_PAYLOAD_MASK;
    s.in = w[LKW_W_IN] & LKW_PAYLOAD_MASK;
    s.out = w[LKW_W_OUT] & LKW_PAYLOAD_MASK;
    s.in2 = w[LKW_W_AUX] & LKW_PAYLOAD_MASK;
    s.a = static_cast<uint32_t>(w[LKW_W_A]);
    s.b = static_cast<uint32_t>(w[LKW_W_B]);
    if (code == LKW_TO_EXIT) reply = LKW_FROM_EXITED;
    else if (code == LKW_TO_NOP) reply = LKW_FROM_NOP;
    else if (code >= LKW_TO_WORK && code < LKW_TO_WORK + lkd::kOpCount) s.op = code - LKW_TO_WORK;
    else reply = LKW_FROM_ERROR;
    if (s.op == 3 || s.op == 7) s.b = static_cast<uint32_t>(w[LKW_W_ALPHA]);
    if (s.op == lkd::kOpBatch) {
      // claim tiles from the shared counter until the table is exhausted
      auto *tiles = reinterpret_cast<const lkd::Tile *>(s.in);
      auto *parts = reinterpret_cast<int64_t *>(s.out);
      auto *counter = reinterpret_cast<uint64_t *>(s.in2);
      const uint64_t base = static_cast<uint64_t>(s.a) | (static_cast<uint64_t>(s.b) << 32);
      for (;;) {
        const uint64_t t = __atomic_fetch_add(counter, 1ull, __ATOMIC_ACQ_REL) - base;
        if (t >= s.n) break;
        const lkd::Tile &tl = tiles[t];
        Slice ts{};
        ts.op = (tl.op == lkd::kOpBatch || tl.op >= lkd::kOpCount) ? 0u : tl.op;
        ts.n = tl.n;
        ts.in = tl.in;
        ts.out = tl.out;
        ts.in2 = tl.in2;
        ts.a = static_cast<uint32_t>(tl.a);
        ts.b = tl.b;
        __atomic_store_n(parts + t, run_slice(ts), __ATOMIC_RELAXED);
        ++partial;
      }
    } else if (reply != LKW_FROM_EXITED) {
      const uint32_t dflags = static_cast<uint32_t>(w[LKW_W_B] >> 32) & 0xffffu;
      // ops: 1 AFFINE_SUM_I32, 2 SUM_I32_I64 (reads x only), 3 SAXPY_F32, 7 AXPY_F32 (y = in2)
      const uint64_t o = s.op == 2 ? 0 : s.out;
      const uint64_t y = s.op == 7 ? s.in2 : 0;
      if ((dflags & (LKW_DF_PIN_INPUT | LKW_DF_PIN_RELOAD)) && (s.op == 1 || s.op == 2 || s.op == 3 || s.op == 7) &&
          s.n > 0 && s.n % 4 == 0 && s.n * 4 <= p.lds_bytes && ((s.in | o | y) & 15u) == 0) {
        PinSlot *hit = nullptr;
        for (PinSlot &e : pins)
          if (e.addr == s.in && e.n == s.n) hit = &e;
        if (!hit || (dflags & LKW_DF_PIN_RELOAD)) {
          if (!hit) {
            const uint64_t used = pins.empty() ? 0 : pins.back().off + pins.back().n;
            if (pins.size() == LKW_PIN_SLOTS || (used + s.n) * 4 > p.lds_bytes) pins.clear();
            const uint64_t off = pins.empty() ? 0 : pins.back().off + pins.back().n;
            pins.push_back(PinSlot{s.in, s.n, off});
            hit = &pins.back();
          }
          memcpy(lds.data() + hit->off, reinterpret_cast<const void *>(s.in), s.n * 4);
        }
        s.in = reinterpret_cast<uint64_t>(lds.data() + hit->off);
      }
      partial = run_slice(s);
      if (s.in2 && (s.op == 1 || s.op == 2)) __atomic_store_n(reinterpret_cast<int64_t *>(s.in2), partial, __ATOMIC_RELAXED);
    }
    const uint64_t t_done = wall_ticks();
    if (p.log && reply != LKW_FROM_EXITED) {
      lkw_log *e = p.log + static_cast<uint64_t>(m) * p.log_cap + (seq % p.log_cap);
      e->seq = static_cast<uint32_t>(want);
      e->code = static_cast<uint16_t>(code);
      e->mailbox = static_cast<uint16_t>(m);
      e->xcc = xcc;
      e->hwid = hw;
      e->t_pick = t_pick;
      e->t_done = t_done;
    }
    // status record: tagged words first, word 0 last with release
    lkw_status *st = sring + slot;
    const uint64_t tag = LKW_TAG(want);
    const uint64_t up = static_cast<uint64_t>(partial);
    st_rlx(&st->w[LKW_S_PART_LO], tag | (up & 0xffffffffull));
    st_rlx(&st->w[LKW_S_PART_HI], tag | (up >> 32));
    st_rlx(&st->w[LKW_S_T_PICK], tag | (t_pick & LKW_PAYLOAD_MASK));
    st_rlx(&st->w[LKW_S_T_DONE], tag | (t_done & LKW_PAYLOAD_MASK));
    st_rlx(&st->w[LKW_S_HWID], tag | hw | (static_cast<uint64_t>(xcc) << 32));
    st_rlx(&st->w[6], tag);
    st_rlx(&st->w[7], tag);
    st_rel(&st->w[LKW_S_WORD], LKW_WORD(want, reply));
    seq = want;
    if (reply == LKW_FROM_EXITED) {
      __atomic_store_n(&wr->t_exit, wall_ticks(), __ATOMIC_RELAXED);
      st_rel(&wr->word, LKW_WORD(want, LKW_FROM_EXITED));
      break;
    }
  }
  running->fetch_sub(1, std::memory_order_release);
}

class FakeDispatch final : public lkbe::Dispatch {
 public:
  bool start(const lkw_params &p, uint32_t n_groups, uint32_t, uint32_t, std::string *) override {
    started_ = clk::now();
    running_.store(n_groups, std::memory_order_relaxed);
    for (uint32_t wg = 0; wg < n_groups; ++wg) th_.emplace_back(worker, p, wg, &running_);
    launched_ = true;
    return true;
  }
  bool finished() const override { return !launched_ || running_.load(std::memory_order_acquire) == 0; }
  double kernel_ms() const override {
    return std::chrono::duration<double, std::milli>(clk::now() - started_).count();
  }
  ~FakeDispatch() override {
    for (auto &t : th_) t.join();
  }

 private:
  std::vector<std::thread> th_;
  std::atomic<uint32_t> running_{0};
  bool launched_ = false;
  clk::time_point started_;
};

}  // namespace

extern "C" void lkfake_freeze(int mailbox) { g_frozen.store(mailbox, std::memory_order_relaxed); }

namespace lkbe {

int device_info(int device, DeviceInfo *out, std::string *err) {
  if (device != 0) {
    *err = "fake device: only device 0";
    return LK_EINVAL;
  }
  const char *e = getenv("LKFAKE_CUS");
  out->cu_count = e ? static_cast<uint32_t>(atoi(e)) : 16u;
  if (out->cu_count == 0 || out->cu_count % 8 != 0) {
    *err = "fake device: the CU count must be a multiple of 8 (8 fake XCDs)";
    return LK_ENODEV;
  }
  out->xcc_count = 8;
  out->lds_per_cu = 160u * 1024u;
  out->wall_hz = 100000000ull;
  return LK_OK;
}

int host_alloc(int, size_t bytes, void **p, std::string *err) {
  *p = aligned_alloc(4096, (bytes + 4095) / 4096 * 4096);
  if (!*p) {
    *err = "out of memory";
    return LK_EHIP;
  }
  memset(*p, 0, bytes);
  return LK_OK;
}
void host_free(void *p) { free(p); }
int device_alloc(int d, size_t bytes, void **p, std::string *err) { return host_alloc(d, bytes, p, err); }
void device_free(void *p) { free(p); }
int device_to_host(void *dst, const void *src, size_t bytes, std::string *) {
  memcpy(dst, src, bytes);
  return LK_OK;
}
Dispatch *open_dispatch(int, std::string *) { return new FakeDispatch(); }

}  // namespace lkbe
