// Kernel launches that can carry per-launch timing events. A measurement hook
// (KTimer in run.hpp) places a pair of events in launch_events() around one
// launcher call; the launcher's kernel is then dispatched with those events
// attached to the dispatch itself, so they time the kernel's execution.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.hpp"

namespace ipcs {

struct LaunchEvents {
  hipEvent_t start, stop;
};

// Per-thread slot read (and cleared) by the next launch().
LaunchEvents*& launch_events();

template <class... KArgs, class... Args>
inline void launch(void (*kernel)(KArgs...), dim3 grid, dim3 block, uint32_t shmem,
                   hipStream_t s, Args... args) {
  LaunchEvents*& le = launch_events();
  if (le) {
    const LaunchEvents e = *le;
    le = nullptr;
    hipExtLaunchKernelGGL(kernel, grid, block, shmem, s, e.start, e.stop, 0u, args...);
  } else {
    hipLaunchKernelGGL(kernel, grid, block, shmem, s, args...);
  }
  HIP_LAUNCH_OK();
}

}  // namespace ipcs
