// Library-internal helpers: error state, workspace carving, launch checks.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>

#include <string>

#include "../../include/voxcsf.h"

namespace vx {

// Last error message of this host thread.
void set_error(const char* fmt, ...);
const char* get_error();

#define VX_FAIL(code, ...)           \
  do {                               \
    ::vx::set_error(__VA_ARGS__);    \
    return (code);                   \
  } while (0)

#define VX_HIP(call)                                                                          \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess) VX_FAIL(VX_EHIP, "%s failed: %s", #call, hipGetErrorString(e_));    \
  } while (0)

#define VX_CHECK_LAUNCH(what)                                                                 \
  do {                                                                                        \
    hipError_t e_ = hipGetLastError();                                                        \
    if (e_ != hipSuccess) VX_FAIL(VX_EHIP, "launch of %s failed: %s", what, hipGetErrorString(e_)); \
  } while (0)

// Bump allocator over a caller-provided workspace.  With base == nullptr it
// only measures (used by the *_workspace_bytes queries and to check the
// caller's size before any launch).
struct Arena {
  char* base = nullptr;
  size_t size = 0, off = 0;
  bool overflow = false;
  template <class T>
  T* take(size_t count, size_t align = 256) {
    off = (off + align - 1) / align * align;
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    if (base && off > size) overflow = true;
    return p;
  }
};

inline int64_t binom64(int n, int r) {
  if (r < 0 || n < r) return 0;
  int64_t v = 1;
  for (int i = 1; i <= r; i++) v = v * (n - r + i) / i;
  return v;
}

// Number of trailing exponent tuples of dimension m with total degree <= d.
inline int64_t ntup(int m, int d) { return binom64(d + m, m); }

}  // namespace vx
