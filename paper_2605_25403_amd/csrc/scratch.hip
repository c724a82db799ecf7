// The fixed memory behind ipcs_batch_step_noalloc, for callers that cannot
// allocate: a device array with room for the shared-launch descriptors (group
// tables, block maps, polling slots) of one Krylov solve of a batch step, and
// a host array for the status polls. Every GPU the library runs on holds its
// own copy of the device array from the time the library's code object is
// loaded on it until the process ends.
#include <hip/hip_runtime.h>

#include <mutex>

#include "common.hpp"
#include "run.hpp"

namespace ipcs {

namespace {

constexpr size_t kScratchBytes = IPCS_BATCH_SCRATCH_BYTES;
constexpr int kMaxDevices = 16;
constexpr int kHostStates = GMAX * IPCS_BATCH_NOALLOC_MAX_RUNS;

// host staging of the status polls, one array per device
KState host_states[kMaxDevices][kHostStates];

int current_device() {
  int dev = -1;
  HIP_OK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) fail(IPCS_E_DEVICE, "device index out of range");
  return dev;
}

// Host code must not pass this name to a kernel or a copy: on the host it is a
// stand-in, not the device address. batch_scratch() returns the address.
static __device__ __align__(256) char scratch[kScratchBytes];

}  // namespace

char* batch_scratch(size_t* cap) {
  static std::mutex mu;
  static char* addr[kMaxDevices] = {};
  const int dev = current_device();
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    // once per device, with that device current: its copy's address
    void* p = nullptr;
    HIP_OK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) fail(IPCS_E_DEVICE, "no device address for the batch scratch array");
    addr[dev] = static_cast<char*>(p);
  }
  *cap = kScratchBytes;
  return addr[dev];
}

KState* batch_host_staging(int* cap) {
  *cap = kHostStates;
  return host_states[current_device()];
}

}  // namespace ipcs
