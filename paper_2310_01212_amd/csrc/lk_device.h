/*
 * lk_device.h -- internal interface between the host library and the gfx950 kernels.
 */
#ifndef LK_DEVICE_H
#define LK_DEVICE_H

#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include "lk_common.h"
#include "lk_wire.h"

namespace lkd {

// Argument block of the per-launch item kernel (grid = k workgroups).
struct ItemArgs {
  uint32_t op;
  uint32_t k;
  uint64_t n;
  const void *in;
  void *out;
  const void *in2;      // AXPY_F32: y
  uint32_t a, b;
  float alpha;
  uint32_t pad;
  int64_t *aux;         // device, k entries, or null
  int64_t *partials;    // host-coherent, k entries, or null
  uint64_t *done_word;  // host-coherent completion word, or null
  uint64_t done_value;
  uint32_t *counter;    // device counter (k > 1), left at 0 after each launch
};

const void *item_kernel();
hipError_t launch_item(const ItemArgs &a, uint32_t threads, hipStream_t s);
hipError_t launch_pingpong(uint64_t *h2d, uint64_t *d2h, uint32_t stride, uint32_t workers, uint64_t iters,
                           uint64_t deadline_ticks, uint32_t poll_sleep, uint32_t *status, bool spread,
                           hipStream_t s);
// Store policies of the copy probe.
constexpr uint32_t kCopyPlain = 0, kCopyNontemporal = 1, kCopySystem = 2;
hipError_t launch_copy_probe(const void *in, void *out, uint64_t bytes, uint32_t grid, uint32_t threads,
                             uint32_t unroll, uint32_t policy, hipStream_t s);

}  // namespace lkd

#endif
