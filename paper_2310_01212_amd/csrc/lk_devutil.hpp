/*
 * lk_devutil.hpp -- device helpers shared by the gfx950 kernels: hardware-id registers,
 * system-scope loads/stores on fine-grained host-coherent memory, store draining and
 * polling backoff.
 */
#ifndef LK_DEVUTIL_HPP
#define LK_DEVUTIL_HPP

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lkdev {

// Hardware registers (s_getreg): HW_ID is hwreg 4 and XCC_ID hwreg 20 on gfx942/gfx950.
// Size field is size-1, offset field in bits [10:6].
__device__ __forceinline__ uint32_t read_hw_id() { return __builtin_amdgcn_s_getreg((31 << 11) | (0 << 6) | 4); }
__device__ __forceinline__ uint32_t read_xcc_id() { return __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20); }

__device__ __forceinline__ uint64_t ld_sys(const uint64_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ void st_sys(uint64_t *p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ void st_sys_i64(int64_t *p, int64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ void st_sys_u32(uint32_t *p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ void st_sys_release(uint64_t *p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Wait until every store this wave issued has been acknowledged by the memory system,
// so that a later release by another wave of the workgroup (ordered after a barrier)
// covers them.
__device__ __forceinline__ void drain_wave_memory() { __builtin_amdgcn_s_waitcnt(0); }

__device__ __forceinline__ void backoff(uint32_t units) {
  for (uint32_t i = 0; i < units; ++i) __builtin_amdgcn_s_sleep(1);
}

// Values every lane holds identically (descriptor fields broadcast through LDS): tell the
// compiler so that loop bounds and base addresses live in scalar registers.
__device__ __forceinline__ uint32_t uniform_u32(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t uniform_u64(uint64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v >> 32));
  return (static_cast<uint64_t>(hi) << 32) | lo;
}

}  // namespace lkdev

#endif
