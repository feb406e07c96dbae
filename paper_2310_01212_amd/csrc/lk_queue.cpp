/*
 * lk_queue.cpp -- dispatch of the persistent worker on an HSA queue of its own.
 *
 * The paper spawns one persistent kernel at boot (Sec. 2.3).  Here that single dispatch
 * is an AQL kernel-dispatch packet written by the library into a hardware queue that
 * nothing else uses.  Because the queue is not a HIP stream, no HIP stream semantics can
 * ever wait behind the never-ending dispatch: the legacy default stream, device-wide
 * synchronisation and the runtime's sharing of a few hardware queues among many streams
 * all leave it alone, and any other work keeps flowing on the remaining queues.
 *
 * The worker is compiled to a standalone code object (lk_worker.hsaco, next to the
 * shared library) and loaded with the HSA loader; it takes no implicit kernel argument,
 * so its kernarg segment is exactly lkw_params.
 */
#include "lk_queue.h"

#include <dlfcn.h>
#include <hip/hip_runtime_api.h>
#include <hsa/hsa.h>
#include <hsa/hsa_ext_amd.h>
#include <immintrin.h>

#include <cstdio>
#include <cstring>
#include <fstream>
#include <string>
#include <vector>

namespace lkq {

namespace {

struct AgentPick {
  uint32_t domain, bus, device;
  hsa_agent_t found{0};
  bool ok = false;
};

hsa_status_t pick_agent(hsa_agent_t a, void *data) {
  auto *p = static_cast<AgentPick *>(data);
  hsa_device_type_t t;
  if (hsa_agent_get_info(a, HSA_AGENT_INFO_DEVICE, &t) != HSA_STATUS_SUCCESS || t != HSA_DEVICE_TYPE_GPU)
    return HSA_STATUS_SUCCESS;
  uint32_t bdf = 0, dom = 0;
  hsa_agent_get_info(a, static_cast<hsa_agent_info_t>(HSA_AMD_AGENT_INFO_BDFID), &bdf);
  hsa_agent_get_info(a, static_cast<hsa_agent_info_t>(HSA_AMD_AGENT_INFO_DOMAIN), &dom);
  if (((bdf >> 8) & 0xffu) == p->bus && ((bdf >> 3) & 0x1fu) == p->device && dom == p->domain) {
    p->found = a;
    p->ok = true;
    return HSA_STATUS_INFO_BREAK;
  }
  return HSA_STATUS_SUCCESS;
}

void queue_error(hsa_status_t status, hsa_queue_t *, void *) {
  const char *msg = nullptr;
  hsa_status_string(status, &msg);
  fprintf(stderr, "lk: persistent-worker queue error: %s\n", msg ? msg : "?");
}

std::string here_dir() {
  Dl_info info;
  if (dladdr(reinterpret_cast<void *>(&here_dir), &info) && info.dli_fname) {
    std::string p(info.dli_fname);
    const size_t s = p.rfind('/');
    if (s != std::string::npos) return p.substr(0, s);
  }
  return ".";
}

std::string hsa_msg(hsa_status_t s) {
  const char *m = nullptr;
  hsa_status_string(s, &m);
  return m ? m : "unknown HSA status";
}

}  // namespace

bool Queue::open(int hip_device, std::string &err) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, hip_device) != hipSuccess) {
    err = "hipGetDeviceProperties failed";
    return false;
  }
  hsa_status_t s = hsa_init();
  if (s != HSA_STATUS_SUCCESS) {
    err = "hsa_init: " + hsa_msg(s);
    return false;
  }
  hsa_inited = true;
  AgentPick pick{static_cast<uint32_t>(prop.pciDomainID), static_cast<uint32_t>(prop.pciBusID),
                 static_cast<uint32_t>(prop.pciDeviceID)};
  hsa_iterate_agents(pick_agent, &pick);
  if (!pick.ok) {
    err = "no HSA agent matches the HIP device's PCI address";
    return false;
  }
  agent = pick.found;

  // Code object of the worker.
  const std::string path = here_dir() + "/lk_worker.hsaco";
  std::ifstream f(path, std::ios::binary);
  if (!f) {
    err = "cannot read " + path;
    return false;
  }
  blob.assign(std::istreambuf_iterator<char>(f), std::istreambuf_iterator<char>());
  if ((s = hsa_code_object_reader_create_from_memory(blob.data(), blob.size(), &reader)) != HSA_STATUS_SUCCESS) {
    err = "code object reader: " + hsa_msg(s);
    return false;
  }
  have_reader = true;
  hsa_profile_t profile;
  hsa_agent_get_info(agent, HSA_AGENT_INFO_PROFILE, &profile);
  if ((s = hsa_executable_create_alt(profile, HSA_DEFAULT_FLOAT_ROUNDING_MODE_DEFAULT, nullptr, &exe)) !=
      HSA_STATUS_SUCCESS) {
    err = "executable create: " + hsa_msg(s);
    return false;
  }
  have_exe = true;
  if ((s = hsa_executable_load_agent_code_object(exe, agent, reader, nullptr, nullptr)) != HSA_STATUS_SUCCESS) {
    err = "load code object: " + hsa_msg(s);
    return false;
  }
  if ((s = hsa_executable_freeze(exe, nullptr)) != HSA_STATUS_SUCCESS) {
    err = "freeze: " + hsa_msg(s);
    return false;
  }
  hsa_executable_symbol_t sym;
  if ((s = hsa_executable_get_symbol_by_name(exe, "lk_worker.kd", &agent, &sym)) != HSA_STATUS_SUCCESS) {
    err = "symbol lk_worker.kd: " + hsa_msg(s);
    return false;
  }
  hsa_executable_symbol_get_info(sym, HSA_EXECUTABLE_SYMBOL_INFO_KERNEL_OBJECT, &kernel_object);
  hsa_executable_symbol_get_info(sym, HSA_EXECUTABLE_SYMBOL_INFO_KERNEL_KERNARG_SEGMENT_SIZE, &kernarg_size);
  hsa_executable_symbol_get_info(sym, HSA_EXECUTABLE_SYMBOL_INFO_KERNEL_GROUP_SEGMENT_SIZE, &group_static);
  hsa_executable_symbol_get_info(sym, HSA_EXECUTABLE_SYMBOL_INFO_KERNEL_PRIVATE_SEGMENT_SIZE, &private_size);

  uint32_t qmin = 64, qmax = 4096;
  hsa_agent_get_info(agent, HSA_AGENT_INFO_QUEUE_MIN_SIZE, &qmin);
  hsa_agent_get_info(agent, HSA_AGENT_INFO_QUEUE_MAX_SIZE, &qmax);
  uint32_t qsize = qmin < 64 ? 64 : qmin;
  if (qsize > qmax) qsize = qmax;
  if ((s = hsa_queue_create(agent, qsize, HSA_QUEUE_TYPE_SINGLE, queue_error, nullptr, UINT32_MAX, UINT32_MAX,
                            &queue)) != HSA_STATUS_SUCCESS) {
    err = "hsa_queue_create: " + hsa_msg(s);
    return false;
  }
  hsa_amd_profiling_set_profiler_enabled(queue, 1);
  if ((s = hsa_signal_create(1, 0, nullptr, &done)) != HSA_STATUS_SUCCESS) {
    err = "hsa_signal_create: " + hsa_msg(s);
    return false;
  }
  have_signal = true;
  const size_t kbytes = kernarg_size < 256 ? 256 : (kernarg_size + 255) / 256 * 256;
  if (hipHostMalloc(&kernarg, kbytes, hipHostMallocCoherent | hipHostMallocMapped | hipHostMallocPortable) !=
      hipSuccess) {
    kernarg = nullptr;
    err = "kernarg allocation failed";
    return false;
  }
  memset(kernarg, 0, kbytes);
  hsa_system_get_info(HSA_SYSTEM_INFO_TIMESTAMP_FREQUENCY, &ts_freq);
  return true;
}

bool Queue::dispatch(const lkw_params &p, uint32_t n_groups, uint32_t threads, uint32_t dyn_lds, std::string &err) {
  if (kernarg_size < sizeof(lkw_params)) {
    err = "worker kernarg segment smaller than lkw_params";
    return false;
  }
  memcpy(kernarg, &p, sizeof p);
  const uint64_t idx = hsa_queue_add_write_index_screlease(queue, 1);
  if (idx - hsa_queue_load_read_index_scacquire(queue) >= queue->size) {
    err = "persistent-worker queue full";
    return false;
  }
  auto *pkt = static_cast<hsa_kernel_dispatch_packet_t *>(queue->base_address) + (idx & (queue->size - 1));
  memset(reinterpret_cast<char *>(pkt) + 4, 0, sizeof(*pkt) - 4);
  pkt->workgroup_size_x = static_cast<uint16_t>(threads);
  pkt->workgroup_size_y = 1;
  pkt->workgroup_size_z = 1;
  pkt->grid_size_x = n_groups * threads;
  pkt->grid_size_y = 1;
  pkt->grid_size_z = 1;
  pkt->private_segment_size = private_size;
  pkt->group_segment_size = group_static + dyn_lds;
  pkt->kernel_object = kernel_object;
  pkt->kernarg_address = kernarg;
  pkt->completion_signal = done;
  const uint16_t header = static_cast<uint16_t>((HSA_PACKET_TYPE_KERNEL_DISPATCH << HSA_PACKET_HEADER_TYPE) |
                                                (1u << HSA_PACKET_HEADER_BARRIER) |
                                                (HSA_FENCE_SCOPE_SYSTEM << HSA_PACKET_HEADER_SCACQUIRE_FENCE_SCOPE) |
                                                (HSA_FENCE_SCOPE_SYSTEM << HSA_PACKET_HEADER_SCRELEASE_FENCE_SCOPE));
  const uint16_t setup = 1u << HSA_KERNEL_DISPATCH_PACKET_SETUP_DIMENSIONS;
  __atomic_store_n(reinterpret_cast<uint32_t *>(pkt), header | (static_cast<uint32_t>(setup) << 16), __ATOMIC_RELEASE);
  hsa_signal_store_screlease(queue->doorbell_signal, static_cast<hsa_signal_value_t>(idx));
  dispatched = true;
  return true;
}

bool Queue::finished() const {
  if (!dispatched) return true;
  return hsa_signal_load_scacquire(done) == 0;
}

double Queue::kernel_ms() const {
  if (!dispatched || !finished() || ts_freq == 0) return 0.0;
  hsa_amd_profiling_dispatch_time_t t;
  if (hsa_amd_profiling_get_dispatch_time(agent, done, &t) != HSA_STATUS_SUCCESS) return 0.0;
  return static_cast<double>(t.end - t.start) * 1e3 / static_cast<double>(ts_freq);
}

void Queue::close() {
  if (queue) hsa_queue_destroy(queue);
  queue = nullptr;
  if (have_signal) hsa_signal_destroy(done);
  have_signal = false;
  if (have_exe) hsa_executable_destroy(exe);
  have_exe = false;
  if (have_reader) hsa_code_object_reader_destroy(reader);
  have_reader = false;
  if (kernarg) (void)hipHostFree(kernarg);
  kernarg = nullptr;
  if (hsa_inited) hsa_shut_down();
  hsa_inited = false;
  dispatched = false;
}

}  // namespace lkq
