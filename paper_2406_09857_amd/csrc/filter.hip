// Exclusion filter, bisection and CSF compaction (Algorithm 3 of Moroz,
// arXiv 2406.09857; bisection of G_n into G_2n, Sec. 3.2).
//
// Given a level's CSF S and a keep flag per box:
//   K    = S restricted to the kept boxes; an internal node survives when at
//          least one descendant box does.  Depth by depth from the leaves:
//          newpos_l = exclusive scan of the survival flags, and a node's flag
//          is newpos_{l+1}[ptr[q+1]] > newpos_{l+1}[ptr[q]].
//   next = CSF of the children 2B + c, c in {0,1}^k, of every kept box B.  A
//          depth-(l+1) node of K with label i becomes 2^(l+1) nodes; the
//          children of a copy of node y are the labels 2 i' + b of y's
//          children i' (b = 0, 1), so N_l(next) = 2^l N_l(K) and labels stay
//          ascending under each parent.  Offsets come from a scan of the
//          child counts; every output entry finds its parent by a search
//          staged through LDS, one tile of outputs per workgroup.
// All passes are scans and gathers with one thread per element; nothing
// depends on scheduling order, so the output is deterministic.
#include <hip/hip_runtime.h>
#include <string.h>

#include "common.hpp"
#include "eval.hpp"
#include "fill.hpp"
#include "profile.hpp"
#include "scan.hpp"

namespace vx {

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_tile_sums(int64_t* tile_sum, const int64_t* n_dev,
                                                                  int64_t nmax, int64_t* total_out) {
  (void)n_dev;
  scan_tile_sums_body(tile_sum, scan_tiles(nmax), total_out);
}

struct KeepLoader {
  const uint8_t* keep;
  __device__ int64_t operator()(int64_t i) const { return keep[i] != 0; }
};

struct AnyChildLoader {
  const int32_t* ptr;
  const int32_t* child_pos;
  __device__ int64_t operator()(int64_t i) const { return child_pos[ptr[i + 1]] > child_pos[ptr[i]]; }
};

struct ChildCountLoader {
  const int32_t* src;
  const int32_t* kptr;
  __device__ int64_t operator()(int64_t i) const {
    const int32_t y = src[i];
    return 2 * (int64_t)(kptr[y + 1] - kptr[y]);
  }
};

// Write the kept nodes of one depth.
__global__ void k_compact_level(int64_t n, const int32_t* __restrict__ newpos, const int32_t* __restrict__ idx,
                                const int32_t* __restrict__ ptr, const int32_t* __restrict__ child_newpos,
                                int32_t* __restrict__ kidx, int32_t* __restrict__ kptr,
                                const int64_t* __restrict__ total_child) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && newpos[i + 1] > newpos[i]) {
    const int32_t o = newpos[i];
    kidx[o] = idx[i];
    if (kptr) kptr[o] = child_newpos[ptr[i]];
  }
  if (i == 0 && kptr) kptr[newpos[n]] = (int32_t)*total_child;
}

__global__ void k_next_counts(int k, const int64_t* __restrict__ kcnt, int64_t* __restrict__ ncnt,
                              int64_t* __restrict__ d_counts) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    for (int l = 0; l < k; l++) {
      ncnt[l] = kcnt[l] << (l + 1);
      if (d_counts) {
        d_counts[l] = kcnt[l];
        d_counts[k + l] = ncnt[l];
      }
    }
  }
}

// Depth-1 nodes of next: 2i, 2i+1 for every depth-1 label i of K.
__global__ void k_next_first(const int64_t* __restrict__ ncnt, const int32_t* __restrict__ kidx,
                             int32_t* __restrict__ nidx, int32_t* __restrict__ src) {
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= ncnt[0]) return;
  const int64_t j = o >> 1;
  nidx[o] = 2 * kidx[j] + (int32_t)(o & 1);
  if (src) src[o] = (int32_t)j;
}

// Depth l+1 >= 2 of next: the parent of each tile's first output, then one
// tile of outputs per workgroup.
__global__ void k_fill_partition(const int64_t* __restrict__ ncnt_parent, const int64_t* __restrict__ ncnt,
                                 const int32_t* __restrict__ nptr, int32_t* __restrict__ part) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t ntile = (*ncnt + FILL_TILE - 1) / FILL_TILE;
  if (t <= ntile) fill_partition_at(t, ntile, *ncnt_parent, nptr, part);
}

__global__ __launch_bounds__(FILL_THREADS) void k_next_fill(const int64_t* __restrict__ ncnt_parent,
                                                           const int64_t* __restrict__ ncnt,
                                                           const int32_t* __restrict__ part,
                                                           const int32_t* __restrict__ nptr,
                                                           const int32_t* __restrict__ src_parent,
                                                           const int32_t* __restrict__ kptr,
                                                           const int32_t* __restrict__ kidx,
                                                           int32_t* __restrict__ nidx, int32_t* __restrict__ src) {
  const int64_t n = *ncnt;
  if ((int64_t)blockIdx.x * FILL_TILE >= n) return;
  next_fill_tile(blockIdx.x, n, *ncnt_parent, part, nptr, src_parent, kptr, kidx, nidx, src);
}

// ---------------------------------------------------------------------------
// Small levels: the whole filter in one workgroup (survival scans, compaction,
// counts, next CSF), the same outputs as the multi-launch path below.
// ---------------------------------------------------------------------------
constexpr int64_t SMALL_FILTER_NODES = 4096;

struct SmallFilterJob {
  const int32_t* idx[VX_KMAX];
  const int32_t* ptr[VX_KMAX];
  int64_t n[VX_KMAX];
  int32_t* newpos[VX_KMAX];
  int32_t* kidx[VX_KMAX];
  int32_t* kptr[VX_KMAX];
  int32_t* nidx[VX_KMAX];
  int32_t* nptr[VX_KMAX];
  int32_t* src[VX_KMAX];
  int64_t* kcnt;
  int64_t* ncnt;
  int64_t* d_counts;
};

// out[0..n] = exclusive prefix sums of ld(0..n-1); returns the total (all threads).
template <class Loader>
__device__ int64_t block_scan_to(Loader ld, int64_t n, int32_t* out) {
  int64_t carry = 0;
  for (int64_t base = 0; base < n; base += SCAN_TILE) {
    const int64_t i0 = base + (int64_t)threadIdx.x * SCAN_ITEMS;
    int64_t v[SCAN_ITEMS];
    int64_t sum = 0;
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; j++) {
      v[j] = i0 + j < n ? ld(i0 + j) : 0;
      sum += v[j];
    }
    int64_t tot;
    int64_t run = carry + block_exclusive_scan(sum, tot);
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; j++) {
      if (i0 + j < n) out[i0 + j] = (int32_t)run;
      run += v[j];
    }
    carry += tot;
  }
  if (threadIdx.x == 0) out[n] = (int32_t)carry;
  __syncthreads();
  return carry;
}

__global__ __launch_bounds__(SCAN_THREADS) void k_filter_small(int k, const uint8_t* __restrict__ keep,
                                                               SmallFilterJob J, int want_next) {
  int64_t kc[VX_KMAX] = {0, 0, 0, 0};
  kc[k - 1] = block_scan_to(KeepLoader{keep}, J.n[k - 1], J.newpos[k - 1]);
  for (int l = k - 2; l >= 0; l--)
    kc[l] = block_scan_to(AnyChildLoader{J.ptr[l], J.newpos[l + 1]}, J.n[l], J.newpos[l]);
  for (int l = 0; l < k; l++) {
    const bool inner = l + 1 < k;
    for (int64_t i = threadIdx.x; i < J.n[l]; i += SCAN_THREADS)
      if (J.newpos[l][i + 1] > J.newpos[l][i]) {
        const int32_t o = J.newpos[l][i];
        J.kidx[l][o] = J.idx[l][i];
        if (inner) J.kptr[l][o] = J.newpos[l + 1][J.ptr[l][i]];
      }
    if (inner && threadIdx.x == 0) J.kptr[l][kc[l]] = (int32_t)kc[l + 1];
  }
  int64_t nc[VX_KMAX] = {0, 0, 0, 0};
  for (int l = 0; l < k; l++) nc[l] = kc[l] << (l + 1);
  if (threadIdx.x == 0)
    for (int l = 0; l < k; l++) {
      J.kcnt[l] = kc[l];
      J.ncnt[l] = nc[l];
      if (J.d_counts) {
        J.d_counts[l] = kc[l];
        J.d_counts[k + l] = nc[l];
      }
    }
  if (!want_next) return;
  __syncthreads();
  for (int64_t o = threadIdx.x; o < nc[0]; o += SCAN_THREADS) {
    J.nidx[0][o] = 2 * J.kidx[0][o >> 1] + (int32_t)(o & 1);
    if (k > 1) J.src[0][o] = (int32_t)(o >> 1);
  }
  __syncthreads();
  for (int l = 1; l < k; l++) {
    block_scan_to(ChildCountLoader{J.src[l - 1], J.kptr[l - 1]}, nc[l - 1], J.nptr[l - 1]);
    // one thread per new parent writes its children (2 per kept child)
    for (int64_t P = threadIdx.x; P < nc[l - 1]; P += SCAN_THREADS) {
      const int32_t y = J.src[l - 1][P];
      const int32_t c0 = J.kptr[l - 1][y], c1 = J.kptr[l - 1][y + 1];
      int64_t o = J.nptr[l - 1][P];
      for (int32_t c = c0; c < c1; c++)
        for (int b = 0; b < 2; b++, o++) {
          J.nidx[l][o] = 2 * J.kidx[l][c] + b;
          if (l + 1 < k) J.src[l][o] = c;
        }
    }
    __syncthreads();
  }
}

struct FilterPlan {
  int32_t* newpos[VX_KMAX] = {};
  int64_t* kcnt = nullptr;
  int64_t* ncnt = nullptr;
  int64_t* tiles = nullptr;
  int32_t* kidx[VX_KMAX] = {};
  int32_t* kptr[VX_KMAX] = {};
  int32_t* src[VX_KMAX] = {};
  int32_t* part = nullptr;
};

static void plan_filter(Arena& A, FilterPlan& F, const vx_csf* S, bool own_kept, bool want_next) {
  const int k = S->k;
  int64_t maxn = 1;
  for (int l = 0; l < k; l++) {
    F.newpos[l] = A.take<int32_t>(S->n[l] + 1);
    const int64_t nb = S->n[l] << (l + 1);
    maxn = maxn > nb ? maxn : nb;
  }
  F.kcnt = A.take<int64_t>(VX_KMAX);
  F.ncnt = A.take<int64_t>(VX_KMAX);
  F.tiles = A.take<int64_t>(scan_tiles(maxn));
  if (own_kept)
    for (int l = 0; l < k; l++) {
      F.kidx[l] = A.take<int32_t>(S->n[l] > 0 ? S->n[l] : 1);
      if (l + 1 < k) F.kptr[l] = A.take<int32_t>(S->n[l] + 1);
    }
  if (want_next) {
    for (int l = 0; l + 1 < k; l++) F.src[l] = A.take<int32_t>((S->n[l] << (l + 1)) + 1);
    F.part = A.take<int32_t>(maxn / FILL_TILE + 2);
  }
}

size_t filter_workspace_bytes(const vx_csf* S) {
  Arena A;
  FilterPlan F;
  plan_filter(A, F, S, true, true);
  return A.off + 256;
}

static int filter_body(const vx_csf* S, const uint8_t* keep, vx_csf* kept, vx_csf* next, int64_t* d_counts,
                       void* ws, size_t ws_bytes, hipStream_t st);

int filter_impl(const vx_csf* S, const uint8_t* keep, vx_csf* kept, vx_csf* next, int64_t* d_counts, void* ws,
                size_t ws_bytes, hipStream_t st) {
  const int ps = prof_start("filter_subdivide", (double)S->n[S->k - 1], st);
  const int rc = filter_body(S, keep, kept, next, d_counts, ws, ws_bytes, st);
  prof_stop(ps, st);
  return rc;
}

static int filter_body(const vx_csf* S, const uint8_t* keep, vx_csf* kept, vx_csf* next, int64_t* d_counts,
                       void* ws, size_t ws_bytes, hipStream_t st) {
  const int k = S->k;
  Arena A;
  A.base = reinterpret_cast<char*>(ws);
  A.size = ws_bytes;
  FilterPlan F;
  plan_filter(A, F, S, kept == nullptr, next != nullptr);
  if (A.overflow)
    VX_FAIL(VX_ECAPACITY, "filter_subdivide: workspace of %zu bytes is too small (%zu needed)", ws_bytes, A.off + 256);
  int32_t* const* kidx = kept ? kept->idx : F.kidx;
  int32_t* const* kptr = kept ? kept->ptr : F.kptr;

  int64_t nmax = 0;
  for (int l = 0; l < k; l++) nmax = S->n[l] > nmax ? S->n[l] : nmax;
  if (nmax <= SMALL_FILTER_NODES) {
    SmallFilterJob J;
    memset(&J, 0, sizeof J);
    for (int l = 0; l < k; l++) {
      J.idx[l] = S->idx[l];
      J.ptr[l] = l + 1 < k ? S->ptr[l] : nullptr;
      J.n[l] = S->n[l];
      J.newpos[l] = F.newpos[l];
      J.kidx[l] = kidx[l];
      J.kptr[l] = l + 1 < k ? kptr[l] : nullptr;
      J.nidx[l] = next ? next->idx[l] : nullptr;
      J.nptr[l] = (next && l + 1 < k) ? next->ptr[l] : nullptr;
      J.src[l] = F.src[l];
    }
    J.kcnt = F.kcnt;
    J.ncnt = F.ncnt;
    J.d_counts = d_counts;
    hipLaunchKernelGGL(k_filter_small, dim3(1), dim3(SCAN_THREADS), 0, st, k, keep, J, next ? 1 : 0);
    VX_CHECK_LAUNCH("k_filter_small");
    return VX_OK;
  }

  // Survival scans, leaves first.
  scan_exclusive(KeepLoader{keep}, (const int64_t*)nullptr, S->n[k - 1], F.newpos[k - 1], F.kcnt + (k - 1), F.tiles,
                 st);
  VX_CHECK_LAUNCH("keep scan");
  for (int l = k - 2; l >= 0; l--) {
    scan_exclusive(AnyChildLoader{S->ptr[l], F.newpos[l + 1]}, (const int64_t*)nullptr, S->n[l], F.newpos[l],
                   F.kcnt + l, F.tiles, st);
    VX_CHECK_LAUNCH("survival scan");
  }
  // Compacted K.
  for (int l = 0; l < k; l++) {
    const int64_t n = S->n[l];
    const bool inner = l + 1 < k;
    hipLaunchKernelGGL(k_compact_level, dim3((unsigned)((n + 255) / 256 > 0 ? (n + 255) / 256 : 1)), dim3(256), 0,
                       st, n, (const int32_t*)F.newpos[l], (const int32_t*)S->idx[l],
                       inner ? (const int32_t*)S->ptr[l] : nullptr, inner ? (const int32_t*)F.newpos[l + 1] : nullptr,
                       kidx[l], inner ? kptr[l] : nullptr, inner ? (const int64_t*)(F.kcnt + l + 1) : nullptr);
    VX_CHECK_LAUNCH("k_compact_level");
  }
  hipLaunchKernelGGL(k_next_counts, dim3(1), dim3(64), 0, st, k, (const int64_t*)F.kcnt, F.ncnt, d_counts);
  VX_CHECK_LAUNCH("k_next_counts");
  if (!next) return VX_OK;

  // Children CSF.
  {
    const int64_t bound = S->n[0] << 1;
    hipLaunchKernelGGL(k_next_first, dim3((unsigned)((bound + 255) / 256 > 0 ? (bound + 255) / 256 : 1)), dim3(256),
                       0, st, (const int64_t*)F.ncnt, (const int32_t*)kidx[0], next->idx[0],
                       k > 1 ? F.src[0] : nullptr);
    VX_CHECK_LAUNCH("k_next_first");
  }
  for (int l = 1; l < k; l++) {
    const int64_t pbound = S->n[l - 1] << l;       // next depth-l count bound
    const int64_t bound = S->n[l] << (l + 1);      // next depth-(l+1) count bound
    scan_exclusive(ChildCountLoader{F.src[l - 1], kptr[l - 1]}, (const int64_t*)(F.ncnt + l - 1), pbound,
                   next->ptr[l - 1], (int64_t*)nullptr, F.tiles, st);
    VX_CHECK_LAUNCH("child count scan");
    const int64_t tiles = (bound + FILL_TILE - 1) / FILL_TILE;
    hipLaunchKernelGGL(k_fill_partition, dim3((unsigned)((tiles + 1 + 255) / 256)), dim3(256), 0, st,
                       (const int64_t*)(F.ncnt + l - 1), (const int64_t*)(F.ncnt + l),
                       (const int32_t*)next->ptr[l - 1], F.part);
    VX_CHECK_LAUNCH("k_fill_partition");
    hipLaunchKernelGGL(k_next_fill, dim3((unsigned)(tiles > 0 ? tiles : 1)), dim3(FILL_THREADS), 0, st,
                       (const int64_t*)(F.ncnt + l - 1), (const int64_t*)(F.ncnt + l), (const int32_t*)F.part,
                       (const int32_t*)next->ptr[l - 1], (const int32_t*)F.src[l - 1], (const int32_t*)kptr[l - 1],
                       (const int32_t*)kidx[l], next->idx[l], l + 1 < k ? F.src[l] : nullptr);
    VX_CHECK_LAUNCH("k_next_fill");
  }
  return VX_OK;
}

}  // namespace vx

namespace vx {

// The level-0 CSF of Algorithm 3: the single box (0, ..., 0).
__global__ void k_init_root(int k, int32_t* i0, int32_t* i1, int32_t* i2, int32_t* i3, int32_t* p0, int32_t* p1,
                            int32_t* p2) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int32_t* idx[4] = {i0, i1, i2, i3};
  int32_t* ptr[3] = {p0, p1, p2};
  for (int l = 0; l < k; l++) {
    idx[l][0] = 0;
    if (l + 1 < k) {
      ptr[l][0] = 0;
      ptr[l][1] = 1;
    }
  }
}

int init_root_impl(vx_csf* S, hipStream_t st) {
  hipLaunchKernelGGL(k_init_root, dim3(1), dim3(64), 0, st, S->k, S->idx[0], S->idx[1], S->idx[2], S->idx[3],
                     S->ptr[0], S->ptr[1], S->ptr[2]);
  VX_CHECK_LAUNCH("k_init_root");
  for (int l = 0; l < S->k; l++) S->n[l] = 1;
  return VX_OK;
}

}  // namespace vx
