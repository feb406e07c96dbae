/*
 * lk_backend.h -- everything the host library (lk_host.cpp) asks of the device: its
 * properties, zero-filled host-coherent and device allocations, a device-to-host copy, and
 * the one persistent dispatch of the worker kernel.  liblk.so implements it with HIP and
 * the HSA runtime (lk_backend_hip.cpp).
 */
#ifndef LK_BACKEND_H
#define LK_BACKEND_H

#include <stddef.h>
#include <stdint.h>

#include <string>

#include "lk_wire.h"

namespace lkbe {

struct DeviceInfo {
  uint32_t cu_count;    // compute units
  uint32_t xcc_count;   // XCDs (accelerator complexes), each with its own L2
  uint32_t lds_per_cu;  // bytes of LDS per CU
  uint64_t wall_hz;     // device wall-clock rate
};

// Checks that `device` exists and is a gfx950 whose LDS per CU holds the one-worker
// padding once but not twice; LK_OK, or LK_ENODEV / LK_EINVAL / LK_EHIP with *err set.
int device_info(int device, DeviceInfo *out, std::string *err);
// Fine-grained host-coherent memory (the mailboxes), zero-filled.
int host_alloc(int device, size_t bytes, void **p, std::string *err);
void host_free(void *p);
// Device memory, zero-filled.
int device_alloc(int device, size_t bytes, void **p, std::string *err);
void device_free(void *p);
int device_to_host(void *dst, const void *src, size_t bytes, std::string *err);

// The persistent dispatch.
class Dispatch {
 public:
  virtual ~Dispatch() = default;
  // One launch of n_groups workgroups of `threads`, each with dyn_lds bytes of LDS on
  // top of the kernel's own (p.n_workers of them become workers; any others leave at boot).
  virtual bool start(const lkw_params &p, uint32_t n_groups, uint32_t threads, uint32_t dyn_lds,
                     std::string *err) = 0;
  // True once the launch has ended (or if there was none).
  virtual bool finished() const = 0;
  // Duration of the ended launch from the dispatcher's timestamps (0 if unknown).
  virtual double kernel_ms() const = 0;
};
// nullptr (and *err) on failure.  Delete only once finished().
Dispatch *open_dispatch(int device, std::string *err);

}  // namespace lkbe

#endif
