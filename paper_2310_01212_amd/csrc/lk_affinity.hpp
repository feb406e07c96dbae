/*
 * lk_affinity.hpp -- pinning of the library's host threads (feeders, schedulers) to
 * distinct CPUs of the process's affinity set, so that threads polling mailboxes keep
 * their cache lines and are not migrated mid-run.
 */
#ifndef LK_AFFINITY_HPP
#define LK_AFFINITY_HPP

#include <pthread.h>
#include <sched.h>

#include <cstddef>
#include <vector>

namespace lkaff {

// CPUs the process may run on, in ascending order (its affinity mask at first use).
inline const std::vector<int> &allowed_cpus() {
  static const std::vector<int> cpus = [] {
    std::vector<int> v;
    cpu_set_t set;
    if (sched_getaffinity(0, sizeof set, &set) == 0)
      for (int i = 0; i < CPU_SETSIZE; ++i)
        if (CPU_ISSET(i, &set)) v.push_back(i);
    return v;
  }();
  return cpus;
}

// Pin the calling thread to the i-th allowed CPU (no-op past the end of the set).
inline void pin_to_allowed_cpu(size_t i) {
  const std::vector<int> &cpus = allowed_cpus();
  if (i >= cpus.size()) return;
  cpu_set_t one;
  CPU_ZERO(&one);
  CPU_SET(cpus[i], &one);
  (void)pthread_setaffinity_np(pthread_self(), sizeof one, &one);
}

}  // namespace lkaff

#endif
