/*
 * lk_device.hip -- gfx950 kernels of the LightKernel dispatch library launched through
 * the HIP runtime (the persistent worker itself is in lk_worker.hip):
 *   lk_item        the same work-item bodies as one ordinary launch per item (the
 *                  "traditional" spawn path the paper compares against, Sec. 3);
 *   lk_pingpong    bare host<->device echo over host-coherent memory: the latency floor
 *                  of any mailbox round trip;
 *   lk_copy_probe  plain streaming copy: the achievable HBM bandwidth, and the known-size
 *                  reference for memory-traffic counters.
 * Every loop that waits on the host is bounded by a device wall-clock deadline.
 */
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "lk_devutil.hpp"
#include "lk_device.h"
#include "lk_ops.hpp"
#include "lk_scratch.h"
#include "lk_wire.h"

using namespace lkdev;

// ----------------------------------------------------------------------------- per-item
// One ordinary launch per item: workgroup j runs slice j of k (same slicing rule and
// same op bodies as the persistent path).  Completion is observed either by stream
// synchronisation or through done_word in host-coherent memory, written by the last
// workgroup to finish.
__global__ void __launch_bounds__(1024) lk_item(lkd::ItemArgs a) {
  __shared__ int64_t s_red[lkops::kMaxWaves];
  const uint32_t j = blockIdx.x;
  uint64_t lo, hi;
  lkd::slice_bounds(a.n, a.k, j, &lo, &hi);
  lkops::Slice s;
  s.op = a.op;
  s.n = hi - lo;
  const uint32_t esz = 4;
  s.in = a.in ? static_cast<const char *>(a.in) + lo * esz : nullptr;
  s.out = a.out ? static_cast<char *>(a.out) + lo * esz : nullptr;
  s.in2 = a.in2 ? static_cast<const char *>(a.in2) + lo * esz : nullptr;
  s.a = a.a;
  s.b = a.b;
  s.alpha = a.alpha;
  const int64_t partial = lkops::run_slice<lkops::CachedStore>(s, s_red, blockDim.x);
  drain_wave_memory();
  __syncthreads();
  if (threadIdx.x == 0) {
    if (a.aux) a.aux[j] = partial;
    if (a.partials) st_sys_i64(a.partials + j, partial);
    // Completion word: written once by the last workgroup to finish, found through the
    // counter (which the launcher guarantees whenever done_word is set and k > 1).
    if (a.done_word) {
      uint32_t last = 1;
      if (a.k > 1) {
        const uint32_t prev = __hip_atomic_fetch_add(a.counter, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        last = prev == a.k - 1;
        if (last) __hip_atomic_store(a.counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      if (last) st_sys_release(a.done_word, a.done_value);
    }
  }
}

// ----------------------------------------------------------------------------- static scratch
// Per-workgroup partial results of the allocation-free per-launch path.  Each GPU the
// library runs on holds its own copy until the process ends.  In host code the array's
// name is not a device address: the address comes from hipGetSymbolAddress, once per
// device (static_partials below), and only that address is handed to kernels or copies.
static __device__ __align__(256) int64_t scratch[lkd::kStaticMaxK];

// ----------------------------------------------------------------------------- probes
// Echo: workgroup w (lane 0) waits for h2d[w*stride] to reach the next value and echoes
// it to d2h[w*stride]; ends after `iters` echoes or when the deadline passes.
__global__ void lk_pingpong(uint64_t *h2d, uint64_t *d2h, uint32_t stride, uint64_t iters,
                            uint64_t deadline_ticks, uint32_t poll_sleep, uint32_t *status) {
  extern __shared__ uint64_t lds_reserve[];
  (void)lds_reserve;
  if (threadIdx.x != 0) return;
  const uint32_t w = blockIdx.x;
  uint64_t *in = h2d + static_cast<uint64_t>(w) * stride;
  uint64_t *out = d2h + static_cast<uint64_t>(w) * stride;
  const uint64_t start = wall_clock64();
  uint64_t expect = 1;
  uint32_t polls = 0;
  while (expect <= iters) {
    const uint64_t v = ld_sys(in);
    if (v >= expect) {
      st_sys(out, v);
      expect = v + 1;
      continue;
    }
    if ((++polls & 255u) == 0 && wall_clock64() - start > deadline_ticks) {
      status[w] = 2;
      return;
    }
    backoff(poll_sleep);
  }
  status[w] = 1;
}

// Streaming copy of nvec 16-byte vectors, grid-stride, U vectors in flight per thread.
// Store policy P: kCopyPlain (ordinary loads and stores), kCopyNontemporal (non-temporal
// loads and stores) or kCopySystem (ordinary loads, stores written through the XCD's L2
// with cache policy sc0 sc1, as the persistent worker writes its outputs; the host keeps
// the output under 2 GiB so that one buffer resource with 32-bit offsets covers it).
template <int U, int P>
__global__ void __launch_bounds__(1024) lk_copy_probe(const lkops::u32x4 *__restrict__ in,
                                                      lkops::u32x4 *__restrict__ out, uint64_t nvec) {
  const uint64_t nt = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  uint64_t k = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const lkops::SystemStore sys(out, P == lkd::kCopySystem ? nvec * 16 : 0);
  auto put = [&](uint64_t i, lkops::u32x4 v) {
    if (P == lkd::kCopyNontemporal) {
      __builtin_nontemporal_store(v, out + i);
    } else if (P == lkd::kCopySystem) {
      sys.put(out + i, v);
    } else {
      out[i] = v;
    }
  };
  for (; k + (U - 1) * nt < nvec; k += U * nt) {
    lkops::u32x4 r[U];
#pragma unroll
    for (int u = 0; u < U; ++u) r[u] = P == lkd::kCopyNontemporal ? __builtin_nontemporal_load(in + k + u * nt) : in[k + u * nt];
#pragma unroll
    for (int u = 0; u < U; ++u) put(k + u * nt, r[u]);
  }
  for (; k < nvec; k += nt) put(k, in[k]);
}

// ----------------------------------------------------------------------------- launchers
namespace lkd {

const void *item_kernel() { return reinterpret_cast<const void *>(lk_item); }

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_addr[kMaxDevices] = {};
}  // namespace

hipError_t static_partials(int device, int64_t **p) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[device]) {
    // the symbol's address on the current device, which the caller has made `device`
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;
    void *q = nullptr;
    e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!q) return hipErrorInvalidSymbol;
    g_scratch_addr[device] = q;
  }
  *p = static_cast<int64_t *>(g_scratch_addr[device]);
  return hipSuccess;
}

hipError_t launch_item(const ItemArgs &a, uint32_t threads, hipStream_t s) {
  // Host-side check of what the kernel assumes: k workgroups (one slice each), a counter
  // whenever more than one workgroup must agree on who writes the completion word, and
  // the pointers every op reads or writes.
  if (a.k == 0 || threads == 0 || threads > 1024 || threads % 64) return hipErrorInvalidValue;
  if (a.done_word && a.k > 1 && !a.counter) return hipErrorInvalidValue;
  const bool reads = a.op == 1 || a.op == 2 || a.op == 3 || a.op == 4 || a.op == 7;
  const bool writes = a.op == 1 || a.op == 3 || a.op == 4 || a.op == 7;
  if (a.op >= kOpCount || a.op == kOpBatch) return hipErrorInvalidValue;
  if (a.n && ((reads && !a.in) || (writes && !a.out) || (a.op == 7 && !a.in2))) return hipErrorInvalidValue;
  hipLaunchKernelGGL(lk_item, dim3(a.k), dim3(threads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_pingpong(uint64_t *h2d, uint64_t *d2h, uint32_t stride, uint32_t workers, uint64_t iters,
                           uint64_t deadline_ticks, uint32_t poll_sleep, uint32_t *status, bool spread,
                           hipStream_t s) {
  uint32_t lds = 0;
  if (spread) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(lk_pingpong),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, LKW_LDS_PAD_BYTES);
    if (e != hipSuccess) return e;
    lds = LKW_LDS_PAD_BYTES;
  }
  hipLaunchKernelGGL(lk_pingpong, dim3(workers), dim3(64), lds, s, h2d, d2h, stride, iters, deadline_ticks,
                     poll_sleep, status);
  return hipGetLastError();
}

hipError_t launch_copy_probe(const void *in, void *out, uint64_t bytes, uint32_t grid, uint32_t threads,
                             uint32_t unroll, uint32_t policy, hipStream_t s) {
  // Host-side check of what the kernel assumes: whole 16-byte vectors, a workgroup of
  // whole waves, and (written-through stores) an output one 32-bit-offset resource covers.
  if (bytes % 16 || grid == 0 || threads == 0 || threads > 1024 || threads % 64) return hipErrorInvalidValue;
  if (policy > kCopySystem || (policy == kCopySystem && bytes >= (1ull << 31))) return hipErrorInvalidValue;
  const auto *src = static_cast<const lkops::u32x4 *>(in);
  auto *dst = static_cast<lkops::u32x4 *>(out);
  const uint64_t nvec = bytes / 16;
#define LKD_COPY(U, P) hipLaunchKernelGGL((lk_copy_probe<U, P>), dim3(grid), dim3(threads), 0, s, src, dst, nvec)
#define LKD_COPY_U(P)                   \
  switch (unroll) {                     \
    case 4: LKD_COPY(4, P); break;      \
    case 8: LKD_COPY(8, P); break;      \
    case 16: LKD_COPY(16, P); break;    \
    default: return hipErrorInvalidValue; \
  }
  switch (policy) {
    case kCopyPlain: LKD_COPY_U(kCopyPlain); break;
    case kCopyNontemporal: LKD_COPY_U(kCopyNontemporal); break;
    default: LKD_COPY_U(kCopySystem); break;
  }
#undef LKD_COPY_U
#undef LKD_COPY
  return hipGetLastError();
}

}  // namespace lkd
