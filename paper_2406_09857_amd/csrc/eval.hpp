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
// Covers eval_level_bytes of every CSF whose node counts are <= S->n.
size_t eval_level_bytes_bound(const vx_poly* P, int np, const vx_csf* S);
// centre = 1 evaluates at the cell centres (degenerate boxes) instead of the
// cells, 2 at the grid vertices; axis_modes (k entries), if given, sets that
// choice per axis instead.
// alive (may be null; S->n[k-2] bytes, k >= 2): the leaf also records, for
// every depth-(k-2) node, whether one of its boxes keeps keep != 0 (the
// survival flag the filter would derive from keep), as long as nothing
// changes keep afterwards.
int eval_level_prepared(const Prepared& Q, const vx_csf* S, const double* dom, double* lo, double* hi, uint8_t* keep,
                        void* ws, size_t ws_bytes, hipStream_t st, const vx_poly* P, int centre = 0,
                        const int* axis_modes = nullptr, uint8_t* alive = nullptr);
// The tables of polynomials idx[0..n) of Q, as a system of their own.
Prepared prepared_subset(const Prepared& Q, const int* idx, int n);

size_t eval_workspace_bytes(const vx_poly* P, int np, const vx_csf* S);
int eval_level_impl(const vx_poly* P, int np, const vx_csf* S, const double* dom, double* lo, double* hi,
                    uint8_t* keep, void* ws, size_t ws_bytes, hipStream_t st, int centre = 0);

size_t filter_workspace_bytes(const vx_csf* S);
// d_counts (device-visible, may be null): the kept counts then the next
// counts, written as soon as they are known; then, when flag is not null,
// *flag = flag_value after a system-scope fence (the host may spin on it
// while the rest of the filter still runs).
// alive (may be null): the survival flags of depth k-2 already known (from
// eval_level_prepared with the same keep); the filter then skips deriving them.
int filter_impl(const vx_csf* S, const uint8_t* keep, vx_csf* kept, vx_csf* next, int64_t* d_counts, void* ws,
                size_t ws_bytes, hipStream_t st, int64_t* flag = nullptr, int64_t flag_value = 0,
                const uint8_t* alive = nullptr);

int init_root_impl(vx_csf* S, hipStream_t st);

size_t build_workspace_bytes(int k, int64_t n);
int build_impl(int k, int level, const int32_t* boxes, int64_t n, vx_csf* out, int64_t* d_counts, void* ws,
               size_t ws_bytes, hipStream_t st);

// Taylor-form exclusion tests of order 1 (mean value) and 2 (criteria.hip).
size_t mv_workspace_bytes(const vx_poly* P, int np, const vx_csf* S, int order);
// With `incl` (order 2) the Taylor-based inclusion flags replace the enclosures.
int mv_impl(const vx_poly* P, int np, const vx_csf* S, const double* dom, double* lo, double* hi, uint8_t* keep,
            void* ws, size_t ws_bytes, hipStream_t st, int order, uint8_t* incl = nullptr);
size_t mv_run_workspace(const vx_poly* P, int np, int order);
size_t mv_level_workspace(const vx_poly* P, int np, const vx_csf* S, int order);
void* mv_run_begin(const vx_poly* P, int np, void* ws, size_t bytes, hipStream_t st, int* rc, int order);
int mv_run_level(void* handle, const vx_poly* P, int np, const vx_csf* S, const double* dom, double* lo, double* hi,
                 uint8_t* keep, void* ws, size_t bytes, hipStream_t st);
void mv_run_end(void* handle);

// Newton interval inclusion test for square systems (criteria.hip); kout
// (nleaf x k x 2, may be null) receives the Krawczyk enclosures.
size_t newton_workspace_bytes(const vx_poly* P, int np, const vx_csf* S);
int newton_impl(const vx_poly* P, int np, const vx_csf* S, const double* dom, uint8_t* incl, double* kout, void* ws,
                size_t ws_bytes, hipStream_t st);

// Inclusion criterion C1 (criteria.hip).
size_t inclusion_workspace_bytes(const vx_poly* P, int np, const vx_csf* S);
int inclusion_impl(const vx_poly* P, int np, const vx_csf* S, const double* dom, uint8_t* incl, void* ws,
                   size_t ws_bytes, hipStream_t st);

size_t batch_workspace_bytes(const vx_poly* P, int nsys, int depth, const int64_t* cap);
int batch_create_impl(const vx_poly* P, int nsys, const double* dom, int depth, const int64_t* cap,
                      const vx_batch_tune* tune, int flags, void* ws, size_t ws_bytes, hipStream_t st,
                      vx_batch** out);
int batch_run_impl(vx_batch* H, hipStream_t st);
int batch_result_impl(vx_batch* H, vx_batch_stat* stats, int64_t* need, vx_csf* last, double* lo, double* hi,
                      uint8_t* keep, vx_csf* kept, hipStream_t st);
int batch_autotune_impl(vx_batch* H, const vx_batch_tune* cand, int ncand, int reps, vx_batch_tune* chosen,
                        float* level_ms, hipStream_t st);
void batch_destroy_impl(vx_batch* H);

// Node counts of S's boxes under each axis order (orders: host, norders x k;
// counts: host, norders x k); synchronizes the stream.
size_t order_workspace_bytes(const vx_csf* S);
int order_counts_impl(const vx_csf* S, int norders, const int32_t* orders, int64_t* counts, void* ws,
                      size_t ws_bytes, hipStream_t st);

}  // namespace vx
