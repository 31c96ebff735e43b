// csf_build: the CSF of an arbitrary list of grid boxes (Sec. 2.1 of Moroz,
// arXiv 2406.09857): depth-l nodes are the distinct prefixes of length l,
// children ascending.
//
// 1. Each box becomes a 64-bit key, labels concatenated (axis 1 most
//    significant), so lexicographic order of boxes = numeric order of keys.
// 2. Stable LSD radix sort, 8-bit digits.  Per pass: per-tile digit
//    histograms, one exclusive scan over (digit, tile), then a stable
//    scatter in which each wave ranks its 64 keys by matching digits with
//    eight ballots (lanes with equal digits, rank = lanes before it), tiles
//    processed in key order.  No atomics decide any position.
// 3. Depth by depth, a node starts where the key's prefix differs from the
//    previous key's; exclusive scans of those flags give every node's index,
//    its label and the offset of its first child.
#include <hip/hip_runtime.h>
#include <string.h>

#include "common.hpp"
#include "eval.hpp"
#include "scan.hpp"

namespace vx {

constexpr int RS_THREADS = 256;
constexpr int RS_ROUNDS = 4;
constexpr int RS_TILE = RS_THREADS * RS_ROUNDS;  // keys per tile
constexpr int RS_BITS = 8;
constexpr int RS_RADIX = 1 << RS_BITS;

__global__ void k_pack_keys(const int32_t* __restrict__ boxes, int64_t n, int k, int level,
                            uint64_t* __restrict__ keys, int32_t* __restrict__ bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t key = 0;
  bool ok = true;
  for (int j = 0; j < k; j++) {
    const int32_t v = boxes[i * k + j];
    ok = ok && v >= 0 && (int64_t)v < ((int64_t)1 << level);
    key = (key << level) | (uint64_t)(uint32_t)(v & ((1u << level) - 1u));
  }
  keys[i] = key;
  if (!ok) *bad = 1;
}

__global__ __launch_bounds__(RS_THREADS) void k_radix_hist(const uint64_t* __restrict__ keys, int64_t n, int shift,
                                                           int64_t ntiles, int64_t* __restrict__ counts) {
  __shared__ int32_t h[RS_RADIX];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * RS_TILE;
  for (int r = 0; r < RS_ROUNDS; r++) {
    const int64_t i = base + r * RS_THREADS + threadIdx.x;
    if (i < n) atomicAdd(&h[(keys[i] >> shift) & (RS_RADIX - 1)], 1);
  }
  __syncthreads();
  counts[(int64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(RS_THREADS) void k_radix_scatter(const uint64_t* __restrict__ keys, int64_t n, int shift,
                                                              int64_t ntiles, const int64_t* __restrict__ offsets,
                                                              uint64_t* __restrict__ out) {
  __shared__ int64_t base[RS_RADIX];
  __shared__ int32_t wcnt[RS_THREADS / 64][RS_RADIX];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  base[threadIdx.x] = offsets[(int64_t)threadIdx.x * ntiles + blockIdx.x];
  for (int w = 0; w < RS_THREADS / 64; w++) wcnt[w][threadIdx.x] = 0;
  __syncthreads();
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t tbase = (int64_t)blockIdx.x * RS_TILE;
  for (int r = 0; r < RS_ROUNDS; r++) {
    const int64_t i = tbase + r * RS_THREADS + threadIdx.x;
    const bool act = i < n;
    const uint64_t key = act ? keys[i] : 0;
    const int dg = (int)((key >> shift) & (RS_RADIX - 1));
    uint64_t match = __ballot(act);
#pragma unroll
    for (int b = 0; b < RS_BITS; b++) {
      const uint64_t ones = __ballot((dg >> b) & 1);
      match &= ((dg >> b) & 1) ? ones : ~ones;
    }
    const int rank = __popcll(match & lt);
    if (act && rank == 0) wcnt[wid][dg] = __popcll(match);
    __syncthreads();
    if (act) {
      int64_t pos = base[dg] + rank;
      for (int w = 0; w < wid; w++) pos += wcnt[w][dg];
      out[pos] = key;
    }
    __syncthreads();
    int32_t add = 0;
    for (int w = 0; w < RS_THREADS / 64; w++) {
      add += wcnt[w][threadIdx.x];
      wcnt[w][threadIdx.x] = 0;
    }
    base[threadIdx.x] += add;
    __syncthreads();
  }
}

// A depth-l node (0-based) starts at key i when the first l+1 labels differ
// from key i-1's.
struct PrefixNewLoader {
  const uint64_t* keys;
  int drop;  // low bits below the prefix
  __device__ int64_t operator()(int64_t i) const {
    return i == 0 || (keys[i] >> drop) != (keys[i - 1] >> drop);
  }
};

__global__ void k_build_level(const uint64_t* __restrict__ keys, int64_t n, int drop, int level,
                              const int32_t* __restrict__ pos, const int32_t* __restrict__ child_pos,
                              int32_t* __restrict__ idx, int32_t* __restrict__ ptr,
                              const int64_t* __restrict__ total_child) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && pos[i + 1] > pos[i]) {
    const int32_t q = pos[i];
    idx[q] = (int32_t)((keys[i] >> drop) & ((1ull << level) - 1ull));
    if (ptr) ptr[q] = child_pos[i];
  }
  if (i == 0 && ptr) ptr[pos[n]] = (int32_t)*total_child;
}

__global__ void k_copy_counts(int k, const int64_t* __restrict__ tot, int64_t* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0)
    for (int l = 0; l < k; l++) out[l] = tot[l];
}

struct CountLoader {
  const int64_t* a;
  __device__ int64_t operator()(int64_t i) const { return a[i]; }
};

struct BuildPlan {
  uint64_t* keys[2] = {};
  int64_t* counts = nullptr;
  int64_t* offsets = nullptr;
  int64_t* tiles = nullptr;
  int32_t* pos[VX_KMAX] = {};
  int64_t* tot = nullptr;
  int32_t* bad = nullptr;
  int64_t* d_counts = nullptr;
  int64_t ntiles = 0;
};

static void plan_build(Arena& A, BuildPlan& B, int k, int64_t n) {
  B.ntiles = (n + RS_TILE - 1) / RS_TILE;
  if (B.ntiles < 1) B.ntiles = 1;
  B.keys[0] = A.take<uint64_t>(n > 0 ? n : 1);
  B.keys[1] = A.take<uint64_t>(n > 0 ? n : 1);
  B.counts = A.take<int64_t>(RS_RADIX * B.ntiles);
  B.offsets = A.take<int64_t>(RS_RADIX * B.ntiles + 1);
  const int64_t big = RS_RADIX * B.ntiles > n ? RS_RADIX * B.ntiles : n;
  B.tiles = A.take<int64_t>(scan_tiles(big));
  for (int l = 0; l < k; l++) B.pos[l] = A.take<int32_t>(n + 1);
  B.tot = A.take<int64_t>(VX_KMAX);
  B.bad = A.take<int32_t>(1);
  B.d_counts = A.take<int64_t>(VX_KMAX);
}

size_t build_workspace_bytes(int k, int64_t n) {
  Arena A;
  BuildPlan B;
  plan_build(A, B, k, n);
  return A.off + 256;
}

int build_impl(int k, int level, const int32_t* boxes, int64_t n, vx_csf* out, int64_t* d_counts, void* ws,
               size_t ws_bytes, hipStream_t st) {
  if ((int64_t)k * level > 62)
    VX_FAIL(VX_EUNSUPPORTED, "csf_build: k * level = %d exceeds the 62-bit key", k * level);
  Arena A;
  A.base = reinterpret_cast<char*>(ws);
  A.size = ws_bytes;
  BuildPlan B;
  plan_build(A, B, k, n);
  if (A.overflow)
    VX_FAIL(VX_ECAPACITY, "csf_build: workspace of %zu bytes is too small (%zu needed)", ws_bytes, A.off + 256);
  if (n == 0) {
    for (int l = 0; l < k; l++) out->n[l] = 0;
    if (k > 1) {
      for (int l = 0; l + 1 < k; l++) VX_HIP(hipMemsetAsync(out->ptr[l], 0, sizeof(int32_t), st));
    }
    return VX_OK;
  }
  VX_HIP(hipMemsetAsync(B.bad, 0, sizeof(int32_t), st));
  const unsigned nb = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(k_pack_keys, dim3(nb), dim3(256), 0, st, boxes, n, k, level, B.keys[0], B.bad);
  VX_CHECK_LAUNCH("k_pack_keys");
  const int bits = k * level;
  int cur = 0;
  for (int shift = 0; shift < bits; shift += RS_BITS) {
    hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)B.ntiles), dim3(RS_THREADS), 0, st, (const uint64_t*)B.keys[cur],
                       n, shift, B.ntiles, B.counts);
    VX_CHECK_LAUNCH("k_radix_hist");
    scan_exclusive(CountLoader{B.counts}, (const int64_t*)nullptr, RS_RADIX * B.ntiles, B.offsets, (int64_t*)nullptr,
                   B.tiles, st);
    VX_CHECK_LAUNCH("radix offsets scan");
    hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)B.ntiles), dim3(RS_THREADS), 0, st,
                       (const uint64_t*)B.keys[cur], n, shift, B.ntiles, (const int64_t*)B.offsets, B.keys[1 - cur]);
    VX_CHECK_LAUNCH("k_radix_scatter");
    cur = 1 - cur;
  }
  const uint64_t* keys = B.keys[cur];
  // node flags and positions, depth by depth
  for (int l = 0; l < k; l++) {
    const int drop = level * (k - 1 - l);
    scan_exclusive(PrefixNewLoader{keys, drop}, (const int64_t*)nullptr, n, B.pos[l], B.tot + l, B.tiles, st);
    VX_CHECK_LAUNCH("prefix scan");
  }
  for (int l = 0; l < k; l++) {
    const int drop = level * (k - 1 - l);
    const bool inner = l + 1 < k;
    hipLaunchKernelGGL(k_build_level, dim3(nb), dim3(256), 0, st, keys, n, drop, level, (const int32_t*)B.pos[l],
                       inner ? (const int32_t*)B.pos[l + 1] : nullptr, out->idx[l], inner ? out->ptr[l] : nullptr,
                       inner ? (const int64_t*)(B.tot + l + 1) : nullptr);
    VX_CHECK_LAUNCH("k_build_level");
  }
  int64_t* dc = d_counts ? d_counts : B.d_counts;
  hipLaunchKernelGGL(k_copy_counts, dim3(1), dim3(64), 0, st, k, (const int64_t*)B.tot, dc);
  VX_CHECK_LAUNCH("k_copy_counts");
  int64_t h[VX_KMAX] = {0, 0, 0, 0};
  int32_t hbad = 0;
  VX_HIP(hipMemcpyAsync(h, dc, sizeof(int64_t) * k, hipMemcpyDeviceToHost, st));
  VX_HIP(hipMemcpyAsync(&hbad, B.bad, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  VX_HIP(hipStreamSynchronize(st));
  for (int l = 0; l < k; l++) out->n[l] = h[l];
  if (hbad) VX_FAIL(VX_EINVAL, "csf_build: a label lies outside [0, 2^%d)", level);
  return VX_OK;
}

}  // namespace vx
