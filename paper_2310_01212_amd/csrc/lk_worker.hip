/*
 * lk_worker.hip -- the persistent worker of the LightKernel dispatch loop for gfx950.
 *
 * One workgroup per CU (Sec. 2.3: one block per cluster, pinned at boot; up to four per
 * CU on request), dispatched once for the whole session on an HSA queue of its own (see
 * lk_queue.cpp).  Each workgroup:
 *   1. on an XCD the context uses (all of them unless it names some), claims a mailbox,
 *      reads its physical placement from the HW_ID / XCC_ID registers and announces
 *      THREAD_INIT (Table 1); on any other XCD it leaves at once;
 *   2. polls its to_GPU command slot: wave 0 reads the whole 64-byte slot with lanes 0..7,
 *      with s_sleep backoff and an idle watchdog on the device wall clock (with a ring
 *      deeper than one slot, a command already posted is usually found by the look-ahead
 *      read issued during the previous item instead);
 *   3. on a new command, takes one system-scope acquire and broadcasts the descriptor to
 *      the workgroup through LDS;
 *   4. runs the work item over its slice with all its waves (lk_ops.hpp), reading a
 *      pinned x from its LDS when the descriptor asks for it;
 *   5. every wave drains its own output stores, which are written through to memory
 *      (SystemStore, lk_ops.hpp); after a barrier wave 0 publishes THREAD_FINISHED as one
 *      64-byte status record (Sec. 2.4: the master thread owns the two mailboxes).
 *      Because no output line is left dirty in the L2, publication needs no L2
 *      writeback, which would otherwise serialise the 32 workers of an XCD;
 *   6. loops until THREAD_EXIT (Table 1) or the watchdog.
 * It is compiled to a standalone code object and uses no implicit kernel argument: the
 * thread count travels in lkw_params.
 */
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lk_devutil.hpp"
#include "lk_device.h"
#include "lk_ops.hpp"
#include "lk_wire.h"

using namespace lkdev;

// BATCH: claim tiles one at a time from the shared counter (value - base = tile index)
// until the table is exhausted; every claim past the end is the member's last.  The
// claim is a system-scope atomic so that it is performed at memory, one counter for the
// members on all XCDs whatever their private L2s hold.  The
// claim for the next tile is issued before the current tile runs so that the atomic's
// round trip overlaps the tile's own loads.  Returns (in thread 0) the number of tiles
// this member executed.
// The claimed index travels through two LDS words used in turn (s_next[0] for the first
// tile, then alternating): thread 0 writes the index of iteration i + 1 while a wave that
// fell behind may still be reading that of iteration i, and the barrier that ends every
// iteration keeps thread 0 from coming back to a word before every wave has read it.
__device__ __forceinline__ int64_t run_batch(const lkd::Tile *tiles, uint64_t n_tiles, int64_t *partials,
                                             uint64_t *counter, uint64_t base, int64_t *s_red, uint64_t *s_next,
                                             uint32_t nt) {
  int64_t executed = 0;
  if (threadIdx.x == 0)
    s_next[0] = __hip_atomic_fetch_add(counter, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) - base;
  __syncthreads();
  for (uint32_t par = 0;; par ^= 1u) {
    const uint64_t t = uniform_u64(s_next[par]);
    if (t >= n_tiles) break;
    const lkd::Tile tile = tiles[t];
    uint64_t next = 0;
    if (threadIdx.x == 0) next = __hip_atomic_fetch_add(counter, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    lkops::Slice sl;
    const uint32_t top = uniform_u32(tile.op);
    sl.op = (top == lkd::kOpBatch || top >= lkd::kOpCount) ? 0u : top;  // no nested batches
    sl.n = uniform_u32(tile.n);
    sl.in = reinterpret_cast<const void *>(uniform_u64(tile.in));
    sl.out = reinterpret_cast<void *>(uniform_u64(tile.out));
    sl.in2 = reinterpret_cast<const void *>(uniform_u64(tile.in2));
    sl.a = uniform_u32(static_cast<uint32_t>(tile.a));
    sl.b = uniform_u32(tile.b);
    sl.alpha = __uint_as_float(sl.b);
    const int64_t part = lkops::run_slice<lkops::SystemStore>(sl, s_red, nt);
    if (threadIdx.x == 0) {
      st_sys_i64(partials + t, part);
      s_next[par ^ 1u] = next - base;
    }
    ++executed;
    __syncthreads();
  }
  return executed;
}

// Lanes 0..7 of wave 0 write the eight tagged words of a status record in one store.
// Each lane picks its word with selects, so the wave does not branch per lane.
__device__ __forceinline__ void publish_status(lkw_status *st, uint64_t seq, uint32_t code, int64_t partial,
                                               uint64_t t_pick, uint64_t t_done, uint32_t hw, uint32_t xcc) {
  const uint32_t lane = threadIdx.x;
  const uint64_t tag = LKW_TAG(seq);
  const uint64_t up = static_cast<uint64_t>(partial);
  uint64_t v = tag;
  v = lane == LKW_S_WORD ? LKW_WORD(seq, code) : v;
  v = lane == LKW_S_PART_LO ? (tag | (up & 0xffffffffull)) : v;
  v = lane == LKW_S_PART_HI ? (tag | (up >> 32)) : v;
  v = lane == LKW_S_T_PICK ? (tag | (t_pick & LKW_PAYLOAD_MASK)) : v;
  v = lane == LKW_S_T_DONE ? (tag | (t_done & LKW_PAYLOAD_MASK)) : v;
  v = lane == LKW_S_HWID ? (tag | hw | (static_cast<uint64_t>(xcc & 0xffffu) << 32)) : v;
  st_sys(&st->w[lane], v);
}

// ----------------------------------------------------------------------------- worker
// Marker wave 0 leaves in the doorbell word when the idle watchdog fires: its code field
// (0xff) is no command code, so no posted doorbell can equal it.
constexpr uint64_t kIdleExit = ~0ull;

// The command loop of one worker (mailbox m), compiled once with the look-ahead read and
// once without it, so a depth-1 context runs none of its bookkeeping.
template <bool LOOK>
__device__ __forceinline__ void serve(const lkw_params &p, uint32_t m, float4 *lds_pin, uint64_t *s_pin, uint64_t *s_w,
                                      uint64_t *s_batch_next, int64_t *s_red) {
  const uint32_t tid = threadIdx.x;
  const uint64_t stride = LKW_RING_STRIDE(p.depth);
  lkw_cmd *ring = p.cmd + m * stride;
  lkw_status *sring = p.status + m * stride;
  lkw_worker *wr = p.workers + m;
  lkw_log *wlog = p.log ? p.log + static_cast<uint64_t>(m) * p.log_cap : nullptr;
  uint64_t seq = 0;                                 // last sequence number executed by this worker
  uint32_t slot = p.depth > 1 ? 1u : 0u;            // ring slot of seq + 1, kept without a division
  uint32_t log_i = 0;                               // log entry of seq + 1
  // Pause before the first poll after a completion (wave 0).  Adaptive: a back-to-back
  // command missed by that first read lengthens it by 2 units, one it finds shortens it
  // by 1, so the first read tends to arrive just after the host has posted.
  uint32_t pre = 8;
  // Look-ahead (ring depth > 1): wave 0 reads the next slot while the current item runs,
  // so a command the host has already posted is taken without another host round trip.
  // The read is issued only when the previous item ran for at least p.la_ticks (about a
  // host round trip): the item's completion waits for the read, which then costs nothing
  // extra, while for short items it would delay every completion.  have_next / v_next
  // (wave 0, lanes 0..7: the slot's words) carry a validated command into the next
  // iteration; its acquire has then already been performed.
  constexpr bool look = LOOK;
  bool have_next = false;
  uint64_t v_next = 0;
  uint64_t last_busy = 0;  // pickup to completion of the previous item (wave 0)

  for (;;) {
    const uint64_t want = seq + 1;

    // ---- poll: wave 0 reads the whole 64-byte slot, one 8-byte word per lane 0..7.
    // Pickup time and placement are scalars of wave 0, kept in registers until the
    // status record is written.
    uint64_t t_pick = 0;
    uint32_t hw = 0, xcc = 0;
    if (tid < 64) {
      const uint64_t *src = ring[slot].w;
      const uint64_t tag = want & 0xffffu;
      const uint64_t t0 = wall_clock64();
      uint32_t polls = 0, outcome = 0;
      uint64_t v = v_next;
      if (!have_next && seq > 0) backoff(p.first_delay < 0 ? pre : static_cast<uint32_t>(p.first_delay));
      while (!have_next) {
        if (tid < LKW_CMD_WORDS) v = ld_sys(src + tid);
        bool ok = true;
        if (tid == 0) ok = LKW_SEQ(v) == want;
        else if (tid < LKW_CMD_WORDS) ok = (v >> LKW_TAG_SHIFT) == tag;
        if (__all(ok)) break;
        ++polls;
        if ((polls & 63u) == 0) {
          const uint64_t now = wall_clock64();
          if (now - t0 > p.idle_ticks) {
            outcome = 1;
            break;
          }
          if ((polls & 4095u) == 0 && tid == 0) st_sys(&wr->heartbeat, now);
        }
        backoff(p.poll_sleep);
      }
      if (!have_next) {
        if (p.first_delay < 0 && seq > 0 && outcome == 0 && wall_clock64() - t0 < p.b2b_ticks)
          pre = polls == 0 ? (pre > 0 ? pre - 1 : 0u) : (pre + 2 > 96 ? 96u : pre + 2);
        if (outcome == 0 && !(p.flags & LKW_K_NO_ACQUIRE)) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
      }
      if (tid < LKW_CMD_WORDS) s_w[tid] = (tid == 0 && outcome != 0) ? kIdleExit : v;
      t_pick = wall_clock64();
      hw = read_hw_id();
      xcc = read_xcc_id();
    }
    __syncthreads();

    // All eight command words in one batch of 16-byte LDS reads, then wave-uniform.  Only
    // lane 0 of each wave reads (readfirstlane takes its values): a full-wave read would
    // move 64 copies of the record through the LDS return path, 64 KiB per item for 16
    // waves.
    const ulonglong2 *sw2 = reinterpret_cast<const ulonglong2 *>(s_w);
    ulonglong2 q0 = {0, 0}, q1 = {0, 0}, q2 = {0, 0}, q3 = {0, 0};
    if ((tid & 63u) == 0) {
      q0 = sw2[0];
      q1 = sw2[1];
      q2 = sw2[2];
      q3 = sw2[3];
    }
    const uint64_t w0 = uniform_u64(q0.x);
    if (w0 == kIdleExit) {  // idle watchdog: leave the loop
      if (tid == 0) {
        st_sys(&wr->t_exit, wall_clock64());
        st_sys_release(&wr->word, LKW_WORD(seq, LKW_FROM_TIMEDOUT));
      }
      return;
    }
    const uint32_t code = LKW_CODE(w0);
    if (code == LKW_TO_EXIT) {  // THREAD_EXIT (Table 1)
      if (tid < LKW_S_WORDS) publish_status(sring + slot, want, LKW_FROM_EXITED, 0, t_pick, t_pick, hw, xcc);
      if (tid == 0) {
        drain_wave_memory();
        st_sys(&wr->t_exit, wall_clock64());
        st_sys_release(&wr->word, LKW_WORD(want, LKW_FROM_EXITED));
      }
      return;
    }

    if (tid == 0 && (p.flags & LKW_K_REPORT_WORKING))
      st_sys(&sring[slot].w[LKW_S_WORD], LKW_WORD(want, LKW_FROM_WORKING));

    uint32_t reply = LKW_FROM_FINISHED;
    lkops::Slice s;
    s.op = 0;
    static_assert(LKW_W_DOORBELL == 0 && LKW_W_N == 1 && LKW_W_IN == 2 && LKW_W_OUT == 3 && LKW_W_AUX == 4 &&
                      LKW_W_A == 5 && LKW_W_B == 6 && LKW_W_ALPHA == 7,
                  "command word order");
    s.n = uniform_u64(q0.y & LKW_PAYLOAD_MASK);
    s.in = reinterpret_cast<const void *>(uniform_u64(q1.x & LKW_PAYLOAD_MASK));
    s.out = reinterpret_cast<void *>(uniform_u64(q1.y & LKW_PAYLOAD_MASK));
    s.in2 = reinterpret_cast<const void *>(uniform_u64(q2.x & LKW_PAYLOAD_MASK));
    s.a = uniform_u32(static_cast<uint32_t>(q2.y));
    s.b = uniform_u32(static_cast<uint32_t>(q3.x));
    const uint32_t dflags = uniform_u32(static_cast<uint32_t>(q3.x >> 32) & 0xffffu);
    s.alpha = __uint_as_float(uniform_u32(static_cast<uint32_t>(q3.y)));
    if (code == LKW_TO_NOP) {
      reply = LKW_FROM_NOP;
    } else if (code >= LKW_TO_WORK && code < LKW_TO_WORK + lkd::kOpCount) {
      s.op = code - LKW_TO_WORK;
    } else {
      reply = LKW_FROM_ERROR;
    }
    // Look-ahead read of the next slot, issued before this wave's own data accesses so
    // that it returns while the item runs (vector memory completes in order).
    const uint32_t slot_next = slot + 1 == p.depth ? 0u : slot + 1;
    uint64_t v_ahead = 0;
    // (Not for a batch: its first tile claim would wait behind the read.)
    const bool ahead_read = look && last_busy >= p.la_ticks && s.op != lkd::kOpBatch;  // wave 0's decision
    if (ahead_read && tid < LKW_CMD_WORDS) v_ahead = ld_sys(ring[slot_next].w + tid);

    int64_t partial = 0;
    if (s.op == lkd::kOpBatch) {
      partial = run_batch(static_cast<const lkd::Tile *>(s.in), s.n, static_cast<int64_t *>(s.out),
                          reinterpret_cast<uint64_t *>(const_cast<void *>(s.in2)),
                          static_cast<uint64_t>(s.a) | (static_cast<uint64_t>(s.b) << 32), s_red, s_batch_next,
                          p.threads);
    } else if (s.op != 0) {
      // Pinned input (AXPY forms and the integer ops): x is served from LDS when one of
      // the worker's pinned slices has the same address and length, else loaded and kept:
      // after the other slices while they fit together, else in place of all of them;
      // RELOAD refills a slice in place.  The table (s_pin) is read here by every thread
      // and written by thread 0 after the completion barrier, so no thread can see an
      // entry whose LDS words it has not filled itself.  The shape check repeats the
      // host's so LDS is never addressed past the buffer.
      const uint64_t ia = reinterpret_cast<uint64_t>(s.in);
      const bool axpy_form = s.op == lkd::kOpSaxpy || s.op == lkd::kOpAxpy;
      const bool int_form = s.op == lkd::kOpAffineSum || s.op == lkd::kOpSumI64;
      const float *y = s.op == lkd::kOpAxpy ? static_cast<const float *>(s.in2) : static_cast<const float *>(s.out);
      const uint64_t oa = s.op == lkd::kOpSumI64 ? 0 : reinterpret_cast<uint64_t>(s.out);
      const uint64_t ya = axpy_form ? reinterpret_cast<uint64_t>(y) : 0;
      const bool pin = (dflags & (LKW_DF_PIN_INPUT | LKW_DF_PIN_RELOAD)) && (axpy_form || int_form) && s.n > 0 &&
                       (s.n & 3u) == 0 && s.n * 4 <= p.lds_bytes && ((ia | oa | ya) & 15u) == 0;
      uint32_t found = LKW_PIN_SLOTS, off16 = 0;  // matching slice and its LDS offset (16-byte units)
      uint32_t fill_slot = 0, fill_off = 0;
      bool reset = false;
      if (pin) {
        for (uint32_t k = 0; k < LKW_PIN_SLOTS; ++k) {
          const uint64_t a = uniform_u64(s_pin[2 * k]), w = uniform_u64(s_pin[2 * k + 1]);
          if (found == LKW_PIN_SLOTS && a == ia && static_cast<uint32_t>(w) == s.n) {
            found = k;
            off16 = static_cast<uint32_t>(w >> 32);
          }
        }
        const uint64_t fl = uniform_u64(s_pin[2 * LKW_PIN_SLOTS]);  // fill level (16-byte units) | count << 32
        const uint32_t used = static_cast<uint32_t>(fl), count = static_cast<uint32_t>(fl >> 32);
        if (found < LKW_PIN_SLOTS) {
          fill_slot = found;
          fill_off = off16;
        } else if (count < LKW_PIN_SLOTS && used + s.n / 4 <= p.lds_bytes / 16) {
          fill_slot = count;
          fill_off = used;
        } else {
          reset = true;
        }
      }
      const bool hit = found < LKW_PIN_SLOTS && !(dflags & LKW_DF_PIN_RELOAD);
      float4 *lds_x = lds_pin + (hit ? off16 : fill_off);
      int4 *lds_i = reinterpret_cast<int4 *>(lds_x);
      const int32_t *xi = static_cast<const int32_t *>(s.in);
      int32_t *yi = static_cast<int32_t *>(s.out);
      if (!pin) {
        partial = lkops::run_slice<lkops::SystemStore>(s, s_red, p.threads);
      } else if (axpy_form) {
        if (hit)
          lkops::axpy_pinned<lkops::SystemStore, false>(static_cast<const float *>(s.in), lds_x, y,
                                                        static_cast<float *>(s.out), s.n, s.alpha, p.threads);
        else
          lkops::axpy_pinned<lkops::SystemStore, true>(static_cast<const float *>(s.in), lds_x, y,
                                                       static_cast<float *>(s.out), s.n, s.alpha, p.threads);
      } else {
        int64_t acc;
        if (s.op == lkd::kOpAffineSum)
          acc = hit ? lkops::affine_sum_pinned<true, lkops::SystemStore, false>(xi, lds_i, yi, s.n, s.a, s.b, p.threads)
                    : lkops::affine_sum_pinned<true, lkops::SystemStore, true>(xi, lds_i, yi, s.n, s.a, s.b, p.threads);
        else
          acc = hit ? lkops::affine_sum_pinned<false, lkops::SystemStore, false>(xi, lds_i, nullptr, s.n, 1u, 0u, p.threads)
                    : lkops::affine_sum_pinned<false, lkops::SystemStore, true>(xi, lds_i, nullptr, s.n, 1u, 0u, p.threads);
        partial = lkops::block_sum_i64(acc, s_red, p.threads);
      }
      // A filled slice is recorded by thread 0 in the pending words; it enters the table
      // after the completion barrier, once every thread has done its lookup.
      if (tid == 0 && pin && !hit) {
        s_pin[2 * LKW_PIN_SLOTS + 1] = ia;
        s_pin[2 * LKW_PIN_SLOTS + 2] = (static_cast<uint64_t>(fill_off) << 32) | s.n;
        s_pin[2 * LKW_PIN_SLOTS + 3] = 0x400u | fill_slot | (reset ? 0x100u : 0u) | (found < LKW_PIN_SLOTS ? 0x200u : 0u);
      }
    }

    // ---- complete.  Thread 0 writes the optional per-member partial with a
    // system-coherent store; every wave then waits until all of its stores have been
    // acknowledged, and the barrier orders all of that before the status record.
    if (tid == 0 && s.in2 && (s.op == 1 || s.op == 2))  // ops with an int64 result
      st_sys_i64(reinterpret_cast<int64_t *>(const_cast<void *>(s.in2)), partial);
    drain_wave_memory();
    // A complete next command (doorbell sequence and every word's tag) found by the
    // look-ahead read is taken here, by wave 0 once its own part of the item is done: its
    // acquire then overlaps the other waves' store drain, and the next item starts as
    // soon as this item's status is out.
    bool ahead = false;
    if (look && ahead_read && tid < 64) {
      const uint64_t nseq = want + 1;
      bool ok = true;
      if (tid == 0) ok = LKW_SEQ(v_ahead) == nseq;
      else if (tid < LKW_CMD_WORDS) ok = (v_ahead >> LKW_TAG_SHIFT) == (nseq & 0xffffu);
      ahead = __all(ok);
      if (ahead && !(p.flags & LKW_K_NO_ACQUIRE)) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
    }
    __syncthreads();
    if (tid < 64) {
      const uint64_t t_done = wall_clock64();
      last_busy = t_done - t_pick;
      have_next = ahead;
      v_next = v_ahead;
      const int64_t part0 = static_cast<int64_t>(uniform_u64(static_cast<uint64_t>(partial)));  // thread 0's
      if (tid < LKW_S_WORDS) publish_status(sring + slot, want, reply, part0, t_pick, t_done, hw, xcc);
      if (tid == 0 && wlog) {
        lkw_log *e = wlog + log_i;
        const uint64_t head = static_cast<uint64_t>(static_cast<uint32_t>(want)) |
                              (static_cast<uint64_t>(code & 0xffffu) << 32) | (static_cast<uint64_t>(m & 0xffffu) << 48);
        st_sys(reinterpret_cast<uint64_t *>(e) + 0, head);
        st_sys(reinterpret_cast<uint64_t *>(e) + 1, static_cast<uint64_t>(xcc) | (static_cast<uint64_t>(hw) << 32));
        st_sys(&e->t_pick, t_pick);
        st_sys(&e->t_done, t_done);
      }
      if (tid == 0) {
        // pending word: slot | 0x100 (reset the table first) | 0x200 (refill in place) | 0x400 (valid)
        const uint64_t pend = s_pin[2 * LKW_PIN_SLOTS + 3];
        if (pend & 0x400u) {
          const uint32_t k = static_cast<uint32_t>(pend) & 0xffu;
          const uint64_t entry = s_pin[2 * LKW_PIN_SLOTS + 2];
          const uint64_t need = (entry & 0xffffffffu) / 4;
          if (pend & 0x100u) {
            for (uint32_t j = 0; j < LKW_PIN_SLOTS; ++j) s_pin[2 * j + 1] = 0;
            s_pin[2 * LKW_PIN_SLOTS] = need | (1ull << 32);
          } else if (!(pend & 0x200u)) {
            s_pin[2 * LKW_PIN_SLOTS] += need + (1ull << 32);
          }
          s_pin[2 * k] = s_pin[2 * LKW_PIN_SLOTS + 1];
          s_pin[2 * k + 1] = entry;
          s_pin[2 * LKW_PIN_SLOTS + 3] = 0;
        }
      }
    }
    seq = want;
    slot = slot_next;
    log_i = log_i + 1 == p.log_cap ? 0u : log_i + 1;
  }
}

extern "C" __global__ void __launch_bounds__(1024) lk_worker(lkw_params p) {
  // Dynamic LDS: holds the CU's LDS share and serves as the pinned-input buffer.
  extern __shared__ float4 lds_pin[];
  // Command words broadcast by wave 0; word 0 holds kIdleExit instead of the doorbell
  // when the idle watchdog fired, so one batch of LDS reads tells every wave what to do.
  __shared__ __align__(16) uint64_t s_w[LKW_CMD_WORDS];
  __shared__ uint64_t s_batch_next[2];
  __shared__ uint32_t s_mb;
  __shared__ int64_t s_red[lkops::kMaxWaves];
  // Pinned-slice table: per slot the device address, then length | LDS offset (16-byte
  // units) << 32 (length 0: empty); then the fill level (16-byte units) | count << 32;
  // then the pending entry of the current item (address, length | offset, flags).
  __shared__ uint64_t s_pin[2 * LKW_PIN_SLOTS + 4];
  const uint32_t tid = threadIdx.x;

  // Boot: claim a mailbox (only on an XCD the context uses), record the physical
  // placement, announce INIT (Table 1).
  if (tid == 0) {
    const uint32_t xcc = read_xcc_id();
    const uint32_t m = ((p.xcc_mask >> (xcc & 31u)) & 1u) ? atomicAdd(p.claim, 1u) : ~0u;
    s_mb = m;
    for (uint32_t j = 0; j < 2 * LKW_PIN_SLOTS + 4; ++j) s_pin[j] = 0;
    if (m < p.n_workers) {
      const uint32_t hw = read_hw_id();
      lkw_worker *wr = p.workers + m;
      st_sys_u32(&wr->hwid, hw);
      st_sys_u32(&wr->xcc, xcc);
      st_sys_u32(&wr->wg, blockIdx.x);
      st_sys(&wr->t_boot, wall_clock64());
      st_sys_release(&wr->word, LKW_WORD(0, LKW_FROM_INIT));
    }
  }
  __syncthreads();
  const uint32_t m = s_mb;
  if (m >= p.n_workers) return;

  if (p.depth > 1 && !(p.flags & LKW_K_NO_LOOKAHEAD))
    serve<true>(p, m, lds_pin, s_pin, s_w, s_batch_next, s_red);
  else
    serve<false>(p, m, lds_pin, s_pin, s_w, s_batch_next, s_red);
}
