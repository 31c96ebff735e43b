// Internal interface of the evaluation kernels (eval.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/voxcsf.h"

namespace vx {

constexpr int VX_MAXPOLY = 64;  // polynomials per system

// Coefficient tables of one call, or of a whole subdivision run: per
// polynomial, the stage-1 coefficient layout, the tuple table and the chain
// length tables (device pointers into a workspace).
struct Prepared {
  int k = 0, np = 0, dmax = 0;
  double* packed[VX_MAXPOLY] = {};
  int2* ttab[VX_MAXPOLY] = {};
  int32_t* lens2[VX_MAXPOLY] = {};
  int32_t* lens1[VX_MAXPOLY] = {};
  int32_t* padlist[VX_MAXPOLY] = {};
  int d[VX_MAXPOLY] = {};
};
size_t prepared_bytes(const vx_poly* P, int np);
int prepare_polys(const vx_poly* P, int np, void* ws, size_t ws_bytes, Prepared* out, hipStream_t st);
size_t eval_level_bytes(const vx_poly* P, int np, const vx_csf* S);
int eval_level_prepared(const Prepared& Q, const vx_csf* S, const double* dom, double* lo, double* hi, uint8_t* keep,
                        void* ws, size_t ws_bytes, hipStream_t st, const vx_poly* P);

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
