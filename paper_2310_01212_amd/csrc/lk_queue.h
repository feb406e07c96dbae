/*
 * lk_queue.h -- the persistent worker's own HSA queue (see lk_queue.cpp).
 */
#ifndef LK_QUEUE_H
#define LK_QUEUE_H

#include <hsa/hsa.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "lk_wire.h"

namespace lkq {

struct Queue {
  hsa_agent_t agent{0};
  hsa_queue_t *queue = nullptr;
  hsa_signal_t done{0};
  hsa_executable_t exe{0};
  hsa_code_object_reader_t reader{0};
  uint64_t kernel_object = 0;
  uint32_t group_static = 0, private_size = 0, kernarg_size = 0;
  void *kernarg = nullptr;
  uint64_t ts_freq = 0;
  std::vector<char> blob;
  bool hsa_inited = false, have_reader = false, have_exe = false, have_signal = false, dispatched = false;

  // Find the HSA agent of a HIP device, load lk_worker.hsaco, create the queue.
  bool open(int hip_device, std::string &err);
  // Write the single dispatch packet: n_groups workgroups of `threads`, plus dyn_lds
  // bytes of LDS per workgroup on top of the worker's static LDS.
  bool dispatch(const lkw_params &p, uint32_t n_groups, uint32_t threads, uint32_t dyn_lds, std::string &err);
  // True once the dispatch has completed (or if nothing was dispatched).
  bool finished() const;
  // Duration of the completed dispatch from the packet processor's timestamps.
  double kernel_ms() const;
  // Release everything; only valid once finished().
  void close();
};

}  // namespace lkq

#endif
