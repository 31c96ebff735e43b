// Internal interface of the evaluation kernels (eval.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/voxcsf.h"

namespace vx {

size_t eval_workspace_bytes(const vx_poly* P, int np, const vx_csf* S);
int eval_level_impl(const vx_poly* P, int np, const vx_csf* S, const double* dom, double* lo, double* hi,
                    uint8_t* keep, void* ws, size_t ws_bytes, hipStream_t st);

size_t filter_workspace_bytes(const vx_csf* S);
int filter_impl(const vx_csf* S, const uint8_t* keep, vx_csf* kept, vx_csf* next, int64_t* d_counts, void* ws,
                size_t ws_bytes, hipStream_t st);

int init_root_impl(vx_csf* S, hipStream_t st);

size_t build_workspace_bytes(int k, int64_t n);
int build_impl(int k, int level, const int32_t* boxes, int64_t n, vx_csf* out, int64_t* d_counts, void* ws,
               size_t ws_bytes, hipStream_t st);

}  // namespace vx
