// csf_build: CSF of an arbitrary list of boxes (Sec. 2.1 of Moroz,
// arXiv 2406.09857).
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "eval.hpp"

namespace vx {

size_t build_workspace_bytes(int k, int64_t n) {
  (void)k;
  return (size_t)(n + 1) * 64 + 4096;
}

int build_impl(int k, int level, const int32_t* boxes, int64_t n, vx_csf* out, int64_t* d_counts, void* ws,
               size_t ws_bytes, hipStream_t st) {
  (void)k; (void)level; (void)boxes; (void)n; (void)out; (void)d_counts; (void)ws; (void)ws_bytes; (void)st;
  VX_FAIL(VX_EUNSUPPORTED, "csf_build is not available in this build yet");
}

}  // namespace vx
