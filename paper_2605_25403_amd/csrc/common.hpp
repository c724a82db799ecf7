// Shared host-side helpers: status exceptions, HIP error checks.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>

#include "ipcs.h"

namespace ipcs {

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] inline void fail(int code, const std::string& msg) { throw Error(code, msg); }

#define IPCS_REQUIRE(cond, msg)                                   \
  do {                                                            \
    if (!(cond)) ::ipcs::fail(IPCS_E_INVALID, std::string(msg)); \
  } while (0)

#define HIP_OK(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      ::ipcs::fail(IPCS_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Checks that a kernel launch was accepted (launch configuration errors).
#define HIP_LAUNCH_OK() HIP_OK(hipGetLastError())

inline int64_t div_up(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int64_t align_up(int64_t a, int64_t b) { return div_up(a, b) * b; }

}  // namespace ipcs
