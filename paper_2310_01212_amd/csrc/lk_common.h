/*
 * lk_common.h -- definitions shared by the host library and the gfx950 kernels that need
 * no device headers: op numbering, the batch tile record and the slicing rule.
 */
#ifndef LK_COMMON_H
#define LK_COMMON_H

#include <stdint.h>

namespace lkd {

constexpr uint32_t kOpCount = 8;  // NOP, AFFINE_SUM_I32, SUM_I32_I64, SAXPY_F32, COPY_F32, SPIN, BATCH, AXPY_F32
constexpr uint32_t kOpAffineSum = 1;
constexpr uint32_t kOpSumI64 = 2;
constexpr uint32_t kOpSaxpy = 3;
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
// the per-launch kernel to cut its grid (constexpr, so device code may call it too).
constexpr void slice_bounds(uint64_t n, uint32_t k, uint32_t j, uint64_t *lo, uint64_t *hi) {
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

}  // namespace lkd

#endif
