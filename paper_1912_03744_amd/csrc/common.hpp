// common.hpp -- host-side helpers shared by the ABI translation units:
// thread-local error messages, HIP status checks, device buffers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <string>

#include "adi.h"

namespace adi {

void set_error(const char* fmt, ...);

// Return `code` after recording a formatted message.
inline adi_status fail(adi_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  set_error("%s", buf);
  return code;
}

#define ADI_HIP(call)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      return ::adi::fail(e_ == hipErrorOutOfMemory ? ADI_ENOMEM : ADI_EDEVICE,         \
                         "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_),        \
                         __FILE__, __LINE__);                                          \
  } while (0)

#define ADI_TRY(expr)                 \
  do {                                \
    adi_status s_ = (expr);           \
    if (s_ != ADI_OK) return s_;      \
  } while (0)

#define ADI_CHECK_LAUNCH() ADI_HIP(hipGetLastError())

// Allocate `bytes` of device memory (zero-filled on `stream`).
adi_status dev_alloc(void** p, size_t bytes, hipStream_t stream);
void dev_free(void* p);

inline bool is_fin(double x) { return x == x && x - x == 0.0; }

}  // namespace adi
