/*
 * lk_device.h -- internal interface between the host library and the gfx950 kernels.
 */
#ifndef LK_DEVICE_H
#define LK_DEVICE_H

#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include "lk_wire.h"

namespace lkd {

constexpr uint32_t kOpCount = 8;  // NOP, AFFINE_SUM_I32, SUM_I32_I64, SAXPY_F32, COPY_F32, SPIN, BATCH, AXPY_F32
constexpr uint32_t kOpBatch = 6;
constexpr uint32_t kOpAxpy = 7;

// Tile record of a batch (same layout as lk_tile in lk.h).
struct Tile {
  uint64_t in, out, in2;
  uint32_t n, op;
  int32_t a;
  uint32_t b;
  uint64_t reserved;
};
static_assert(sizeof(Tile) == 48, "tile record is 48 bytes");

// Slicing rule of a cluster item: m = ceil(n/k) rounded up to a multiple of 256 elements,
// slice j = [min(n, j*m), min(n, (j+1)*m)).  Used by the host to cut descriptors and by
// the per-launch kernel to cut its grid.
__host__ __device__ inline void slice_bounds(uint64_t n, uint32_t k, uint32_t j, uint64_t *lo, uint64_t *hi) {
  if (k == 0 || j >= k) {
    *lo = *hi = n;
    return;
  }
  uint64_t m = (n + k - 1) / k;
  m = (m + 255u) & ~static_cast<uint64_t>(255u);
  const uint64_t l = static_cast<uint64_t>(j) * m;
  *lo = l < n ? l : n;
  *hi = l + m < n ? l + m : n;
}

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
hipError_t launch_copy_probe(const void *in, void *out, uint64_t bytes, uint32_t grid, hipStream_t s);

}  // namespace lkd

#endif
