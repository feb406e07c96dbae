/*
 * lk_scratch.h -- the library's static device scratch (lk_device.hip): per-workgroup
 * partial results of the allocation-free per-launch path.
 */
#ifndef LK_SCRATCH_H
#define LK_SCRATCH_H

#include <hip/hip_runtime_api.h>
#include <stdint.h>

namespace lkd {

// Entries of the static partial-result array: one per workgroup of an item.
constexpr uint32_t kStaticMaxK = 4096;

// Device address of the static partial-result array on `device`, which must be the
// current device; resolved once per device and kept for the life of the process.
hipError_t static_partials(int device, int64_t **p);

}  // namespace lkd

#endif
