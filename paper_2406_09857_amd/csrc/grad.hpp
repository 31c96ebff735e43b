// Internal interface of the point-evaluation / adjoint / Newton kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/voxcsf.h"

namespace vx {

constexpr int PMAX_GRAD = 4;     // polynomials per point system
constexpr int MAXDEG_ADJ = 200;  // largest degree of the coefficient adjoint (LDS power tables)

struct AxisDom {
  double lo[VX_KMAX];
  double hi[VX_KMAX];
};

size_t grad_workspace_bytes(const vx_poly* P, int np, const vx_csf* grid, int64_t n);
int grad_impl(const vx_poly* P, int np, const double* x, int64_t n, double* f, double* jac, const double* gbar,
              double* xbar, double* dcoef, const vx_csf* grid, const double* dom, void* ws, size_t ws_bytes, hipStream_t st);
// grid (may be null): x holds the centres of grid's leaves; the first
// evaluation then runs on the grid (checked bit for bit).
int newton_impl(const vx_poly* P, int np, double* x, int64_t n, int steps, double* f, void* ws, size_t ws_bytes,
                hipStream_t st, const vx_csf* grid = nullptr, const double* dom = nullptr);
int centres_impl(const vx_csf* S, const double* dom, double* x, hipStream_t st);

}  // namespace vx
