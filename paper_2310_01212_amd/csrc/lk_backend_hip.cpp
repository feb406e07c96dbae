/*
 * lk_backend_hip.cpp -- the device side of the host library on an MI355X: HIP for device
 * properties and memory, and the worker's own HSA queue (lk_queue.cpp) for the persistent
 * dispatch.
 */
#include "lk_backend.h"

#include <hip/hip_runtime_api.h>

#include <cstring>

#include "lk.h"
#include "lk_queue.h"

namespace lkbe {

namespace {

int hip_error(hipError_t e, const char *what, std::string *err) {
  *err = std::string(what) + ": " + hipGetErrorString(e);
  return LK_EHIP;
}

class HsaDispatch final : public Dispatch {
 public:
  lkq::Queue q;
  bool start(const lkw_params &p, uint32_t n_groups, uint32_t threads, uint32_t dyn_lds, std::string *err) override {
    return q.dispatch(p, n_groups, threads, dyn_lds, *err);
  }
  bool finished() const override { return q.finished(); }
  double kernel_ms() const override { return q.kernel_ms(); }
  ~HsaDispatch() override { q.close(); }
};

}  // namespace

int device_info(int device, DeviceInfo *out, std::string *err) {
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev == 0) {
    *err = std::string("no HIP device (") + hipGetErrorString(e) + ")";
    return LK_ENODEV;
  }
  if (device < 0 || device >= ndev) {
    *err = "device " + std::to_string(device) + " of " + std::to_string(ndev);
    return LK_EINVAL;
  }
  if ((e = hipSetDevice(device)) != hipSuccess) return hip_error(e, "hipSetDevice", err);
  hipDeviceProp_t prop;
  if ((e = hipGetDeviceProperties(&prop, device)) != hipSuccess) return hip_error(e, "hipGetDeviceProperties", err);
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
    *err = "device " + std::to_string(device) + " is " + prop.gcnArchName + "; this library is built for gfx950";
    return LK_ENODEV;
  }
  // The one-worker-per-CU layout relies on LKW_LDS_PAD_BYTES fitting a CU once, not twice.
  if (prop.maxSharedMemoryPerMultiProcessor < LKW_LDS_PAD_BYTES + 4096 ||
      prop.maxSharedMemoryPerMultiProcessor >= 2 * LKW_LDS_PAD_BYTES) {
    *err = "unexpected LDS size " + std::to_string(prop.maxSharedMemoryPerMultiProcessor) + " per CU";
    return LK_ENODEV;
  }
  out->cu_count = static_cast<uint32_t>(prop.multiProcessorCount);
  int nxcc = 0;
  if ((e = hipDeviceGetAttribute(&nxcc, hipDeviceAttributeNumberOfXccs, device)) != hipSuccess || nxcc <= 0 ||
      nxcc > 32 || out->cu_count % static_cast<uint32_t>(nxcc) != 0) {
    *err = "unexpected XCD count " + std::to_string(nxcc) + " for " + std::to_string(out->cu_count) + " CUs";
    return LK_ENODEV;
  }
  out->xcc_count = static_cast<uint32_t>(nxcc);
  out->lds_per_cu = static_cast<uint32_t>(prop.maxSharedMemoryPerMultiProcessor);
  out->wall_hz = 100000000ull;
  int wc_khz = 0;
  if (hipDeviceGetAttribute(&wc_khz, hipDeviceAttributeWallClockRate, device) == hipSuccess && wc_khz > 0)
    out->wall_hz = static_cast<uint64_t>(wc_khz) * 1000ull;
  return LK_OK;
}

int host_alloc(int device, size_t bytes, void **p, std::string *err) {
  hipError_t e = hipSetDevice(device);
  if (e != hipSuccess) return hip_error(e, "hipSetDevice", err);
  if ((e = hipHostMalloc(p, bytes, hipHostMallocCoherent | hipHostMallocMapped | hipHostMallocPortable)) != hipSuccess) {
    *p = nullptr;
    return hip_error(e, "hipHostMalloc(coherent)", err);
  }
  memset(*p, 0, bytes);
  return LK_OK;
}

void host_free(void *p) {
  if (p) (void)hipHostFree(p);
}

int device_alloc(int device, size_t bytes, void **p, std::string *err) {
  hipError_t e = hipSetDevice(device);
  if (e != hipSuccess) return hip_error(e, "hipSetDevice", err);
  if ((e = hipMalloc(p, bytes)) != hipSuccess) {
    *p = nullptr;
    return hip_error(e, "hipMalloc", err);
  }
  if ((e = hipMemset(*p, 0, bytes)) != hipSuccess) {
    (void)hipFree(*p);
    *p = nullptr;
    return hip_error(e, "hipMemset", err);
  }
  return LK_OK;
}

void device_free(void *p) {
  if (p) (void)hipFree(p);
}

int device_to_host(void *dst, const void *src, size_t bytes, std::string *err) {
  const hipError_t e = hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost);
  return e == hipSuccess ? LK_OK : hip_error(e, "hipMemcpy", err);
}

Dispatch *open_dispatch(int device, std::string *err) {
  auto *d = new HsaDispatch();
  if (!d->q.open(device, *err)) {
    delete d;
    return nullptr;
  }
  return d;
}

}  // namespace lkbe
