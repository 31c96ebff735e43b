// Children of the next CSF at one depth (bisection, Sec. 3.2 of Moroz, arXiv
// 2406.09857): output o belongs to the parent P with nptr[P] <= o <
// nptr[P+1]; the parent is a copy of the kept node y = src_parent[P], and o
// is copy (o - nptr[P]) & 1 of y's kept child kptr[y] + (o - nptr[P]) / 2,
// whose label doubles.
//
// One workgroup fills a tile of FILL_TILE consecutive outputs.  A first pass
// (one thread per tile) finds the parent of each tile's first output; every
// parent has at least two children (a kept internal node keeps a child, and
// each child yields two), so a tile meets at most FILL_TILE/2 + 2 parents,
// whose offsets are staged in LDS, and each output searches only there.
// Should a tile ever meet more parents than the LDS holds, its outputs fall
// back to a global search (same result).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vx {

constexpr int FILL_THREADS = 256;
constexpr int FILL_ITEMS = 4;
constexpr int FILL_TILE = FILL_THREADS * FILL_ITEMS;
constexpr int FILL_LDS = FILL_TILE / 2 + 2;

// Last index P in [0, n) with a[P] <= v (a ascending, a[0] <= v).
__device__ __forceinline__ int64_t last_le(const int32_t* __restrict__ a, int64_t n, int64_t v) {
  int64_t lo = 0, hi = n;
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (a[mid] <= v) lo = mid; else hi = mid;
  }
  return lo;
}

// part[t] = parent of output t * FILL_TILE for t < ntile, part[ntile] = the
// last parent.
__device__ __forceinline__ void fill_partition_at(int64_t t, int64_t ntile, int64_t npar,
                                                  const int32_t* __restrict__ nptr, int32_t* __restrict__ part) {
  part[t] = (int32_t)(t < ntile ? last_le(nptr, npar, t * FILL_TILE) : npar - 1);
}

// Called by all FILL_THREADS threads of a workgroup for tile t (t * FILL_TILE < n).
__device__ __forceinline__ void next_fill_tile(int64_t t, int64_t n, int64_t npar, const int32_t* __restrict__ part,
                                               const int32_t* __restrict__ nptr,
                                               const int32_t* __restrict__ src_parent,
                                               const int32_t* __restrict__ kptr, const int32_t* __restrict__ kidx,
                                               int32_t* __restrict__ nidx, int32_t* __restrict__ src) {
  __shared__ int32_t s_ptr[FILL_LDS];
  const int64_t o0 = t * FILL_TILE;
  const int64_t oend = o0 + FILL_TILE < n ? o0 + FILL_TILE : n;
  const int64_t p0 = part[t];
  const int64_t np = (int64_t)part[t + 1] - p0 + 1;  // parents of outputs o0 .. oend-1 lie in p0 .. part[t+1]
  const bool staged = np <= FILL_LDS;
  if (staged)
    for (int64_t i = threadIdx.x; i < np; i += FILL_THREADS) s_ptr[i] = nptr[p0 + i];
  __syncthreads();
#pragma unroll
  for (int r = 0; r < FILL_ITEMS; r++) {
    const int64_t o = o0 + r * FILL_THREADS + threadIdx.x;
    if (o < oend) {
      int64_t P, start;
      if (staged) {
        int lo = 0, hi = (int)np;
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (s_ptr[mid] <= o) lo = mid; else hi = mid;
        }
        P = p0 + lo;
        start = s_ptr[lo];
      } else {
        P = last_le(nptr, npar, o);
        start = nptr[P];
      }
      const int64_t rel = o - start;
      const int32_t y = src_parent[P];
      const int32_t child = kptr[y] + (int32_t)(rel >> 1);
      nidx[o] = 2 * kidx[child] + (int32_t)(rel & 1);
      if (src) src[o] = child;
    }
  }
  __syncthreads();  // s_ptr is reused by the workgroup's next tile
}

}  // namespace vx
