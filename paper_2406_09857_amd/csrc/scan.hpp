// Device-wide exclusive prefix sums with a device-resident length.
//
// Reduce-then-scan in three launches (tile sums, scan of the tile sums in one
// workgroup, rescan of each tile with its offset).  No atomics and no
// inter-workgroup waiting, so the result is deterministic and every launch
// terminates on its own.  The element count may live in device memory (it is
// often produced by the previous kernel on the same stream); the grid is sized
// from a host-side upper bound and surplus workgroups exit at once.
//
// Within a workgroup: wave64 inclusive scans with cross-lane shuffles, one
// LDS slot per wave for the wave totals.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vx {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

__device__ __forceinline__ int64_t wave_inclusive_scan(int64_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    int64_t u = __shfl_up(v, off, 64);
    if (lane >= off) v += u;
  }
  return v;
}

// Exclusive scan of one value per thread across a workgroup of NT threads;
// returns the thread's exclusive prefix and writes the workgroup total to
// `total`.
template <int NT = SCAN_THREADS>
__device__ __forceinline__ int64_t block_exclusive_scan(int64_t v, int64_t& total) {
  __shared__ int64_t wsum[NT / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int64_t inc = wave_inclusive_scan(v);
  if (lane == 63) wsum[wid] = inc;
  __syncthreads();
  int64_t base = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < NT / 64; w++) {
    const int64_t s = wsum[w];
    if (w < wid) base += s;
    tot += s;
  }
  __syncthreads();
  total = tot;
  return base + inc - v;
}

__host__ __device__ inline int64_t scan_tiles(int64_t nmax);

// Pass 2 body: exclusive scan, in place, of nt tile sums by one workgroup,
// SCAN_ITEMS consecutive sums per thread per round; total to *total_out.
__device__ __forceinline__ void scan_tile_sums_body(int64_t* tile_sum, int64_t nt, int64_t* total_out) {
  int64_t carry = 0;
  for (int64_t base = 0; base < nt; base += SCAN_TILE) {
    const int64_t i0 = base + (int64_t)threadIdx.x * SCAN_ITEMS;
    int64_t v[SCAN_ITEMS];
    int64_t s = 0;
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; j++) {
      v[j] = i0 + j < nt ? tile_sum[i0 + j] : 0;
      s += v[j];
    }
    int64_t tot;
    int64_t run = carry + block_exclusive_scan(s, tot);
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; j++) {
      if (i0 + j < nt) tile_sum[i0 + j] = run;
      run += v[j];
    }
    carry += tot;
  }
  if (threadIdx.x == 0 && total_out) *total_out = carry;
}

__device__ __forceinline__ int64_t load_n(const int64_t* n_dev, int64_t nmax) {
  if (!n_dev) return nmax;
  const int64_t n = *n_dev;
  return n < nmax ? n : nmax;
}

// Pass 1: per-tile sums.
template <class Loader>
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_tiles(Loader ld, const int64_t* n_dev, int64_t nmax,
                                                              int64_t* tile_sum) {
  const int64_t n = load_n(n_dev, nmax);
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
  int64_t s = 0;
  if (base < n) {
    const int64_t i0 = base + (int64_t)threadIdx.x * SCAN_ITEMS;
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; j++)
      if (i0 + j < n) s += ld(i0 + j);
  }
  int64_t tot;
  block_exclusive_scan(s, tot);
  if (threadIdx.x == 0) tile_sum[blockIdx.x] = tot;
}

// Pass 2: exclusive scan of the tile sums in one workgroup.
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_tile_sums(int64_t* tile_sum, const int64_t* n_dev,
                                                                  int64_t nmax, int64_t* total_out);

// Pass 3: rescan each tile with its offset; out[i] for i < n, out[n] = total.
template <class Loader, class OutT>
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_write(Loader ld, const int64_t* n_dev, int64_t nmax,
                                                              const int64_t* tile_off, OutT* out) {
  const int64_t n = load_n(n_dev, nmax);
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
  if (base > n) return;
  const int64_t i0 = base + (int64_t)threadIdx.x * SCAN_ITEMS;
  int64_t v[SCAN_ITEMS];
  int64_t s = 0;
#pragma unroll
  for (int j = 0; j < SCAN_ITEMS; j++) {
    v[j] = (i0 + j < n) ? ld(i0 + j) : 0;
    s += v[j];
  }
  int64_t tot;
  int64_t run = block_exclusive_scan(s, tot) + tile_off[blockIdx.x];
#pragma unroll
  for (int j = 0; j < SCAN_ITEMS; j++) {
    if (i0 + j <= n) out[i0 + j] = (OutT)run;
    run += v[j];
  }
}

__host__ __device__ inline int64_t scan_tiles(int64_t nmax) { return (nmax + 1 + SCAN_TILE - 1) / SCAN_TILE; }

// Host launcher: out[0..n] = exclusive prefix sums of ld(0..n-1), out[n] = total,
// *total_out = total (int64, device).  tile_buf needs scan_tiles(nmax) int64s.
template <class Loader, class OutT>
void scan_exclusive(Loader ld, const int64_t* n_dev, int64_t nmax, OutT* out, int64_t* total_out,
                    int64_t* tile_buf, hipStream_t st) {
  const int64_t nt = scan_tiles(nmax);
  hipLaunchKernelGGL(k_scan_tiles<Loader>, dim3((unsigned)nt), dim3(SCAN_THREADS), 0, st, ld, n_dev, nmax, tile_buf);
  hipLaunchKernelGGL(k_scan_tile_sums, dim3(1), dim3(SCAN_THREADS), 0, st, tile_buf, n_dev, nmax, total_out);
  hipLaunchKernelGGL((k_scan_write<Loader, OutT>), dim3((unsigned)nt), dim3(SCAN_THREADS), 0, st, ld, n_dev, nmax,
                     (const int64_t*)tile_buf, out);
}

// Several independent exclusive scans in three launches: out_a[0..n_a] =
// exclusive prefix sums of in_a, out_a[n_a] = total_a = *total[a].  Inputs
// are 0/1 flags (uint8, nonzero counts as 1) or int64 counts; tiles[a] needs
// scan_tiles(n_a) int64s.  The tiles of all arrays share one 1-D grid, so
// no workgroup is launched idle.
constexpr int MSCAN_MAX = 8;

// One 1-D grid over several arrays: array a owns blocks off[a] .. off[a+1]-1,
// n[a] / per_block + 1 of them (at least one, covering elements 0 .. n[a]).
struct DepthBlocks {
  int64_t off[MSCAN_MAX + 1];
  int count;
  // Array of block b and the block's index within it.
  __device__ __forceinline__ int find(int64_t b, int64_t& t) const {
    int a = 0;
#pragma unroll
    for (int i = 1; i < MSCAN_MAX; i++)
      if (i < count && b >= off[i]) a = i;
    t = b - off[a];
    return a;
  }
  unsigned blocks() const { return (unsigned)off[count]; }
};

inline DepthBlocks depth_blocks(const int64_t* n, int count, int64_t per_block) {
  DepthBlocks D;
  D.count = count;
  D.off[0] = 0;
  for (int a = 0; a < MSCAN_MAX; a++) D.off[a + 1] = D.off[a] + (a < count ? n[a] / per_block + 1 : 0);
  return D;
}

template <class In, class Out>
struct MultiScan {
  const In* in[MSCAN_MAX];
  Out* out[MSCAN_MAX];
  int64_t* total[MSCAN_MAX];
  int64_t* tiles[MSCAN_MAX];
  int64_t n[MSCAN_MAX];
  DepthBlocks D;
};

// The SCAN_ITEMS inputs of one thread (consecutive, i0 .. i0+7), 0 past n.
__device__ __forceinline__ void mscan_load(const uint8_t* in, int64_t i0, int64_t n, int64_t* v) {
  if (i0 + SCAN_ITEMS <= n && ((uintptr_t)(in + i0) & 7) == 0) {
    const uint64_t w = *reinterpret_cast<const uint64_t*>(in + i0);
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; j++) v[j] = ((w >> (8 * j)) & 0xff) != 0;
  } else {
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; j++) v[j] = i0 + j < n ? in[i0 + j] != 0 : 0;
  }
}

__device__ __forceinline__ void mscan_load(const int64_t* in, int64_t i0, int64_t n, int64_t* v) {
#pragma unroll
  for (int j = 0; j < SCAN_ITEMS; j++) v[j] = i0 + j < n ? in[i0 + j] : 0;
}

// out[i0 + j] = r[j] for i0 + j <= n.
__device__ __forceinline__ void mscan_store(int32_t* out, int64_t i0, int64_t n, const int64_t* r) {
  if (i0 + SCAN_ITEMS <= n + 1 && ((uintptr_t)(out + i0) & 31) == 0) {
    int4* o = reinterpret_cast<int4*>(out + i0);
    o[0] = make_int4((int)r[0], (int)r[1], (int)r[2], (int)r[3]);
    o[1] = make_int4((int)r[4], (int)r[5], (int)r[6], (int)r[7]);
  } else {
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; j++)
      if (i0 + j <= n) out[i0 + j] = (int32_t)r[j];
  }
}

__device__ __forceinline__ void mscan_store(int64_t* out, int64_t i0, int64_t n, const int64_t* r) {
#pragma unroll
  for (int j = 0; j < SCAN_ITEMS; j++)
    if (i0 + j <= n) out[i0 + j] = r[j];
}

static_assert(SCAN_ITEMS == 8, "the vector paths of mscan_load / mscan_store move 8 items");

template <class In, class Out>
__global__ __launch_bounds__(SCAN_THREADS) void k_mscan_tiles(MultiScan<In, Out> M) {
  int64_t t;
  const int a = M.D.find(blockIdx.x, t);
  const int64_t n = M.n[a];
  const int64_t i0 = t * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  int64_t v[SCAN_ITEMS];
  mscan_load(M.in[a], i0, n, v);
  int64_t sum = 0;
#pragma unroll
  for (int j = 0; j < SCAN_ITEMS; j++) sum += v[j];
  int64_t tot;
  block_exclusive_scan(sum, tot);
  if (threadIdx.x == 0) M.tiles[a][t] = tot;
}

template <class In, class Out>
__global__ __launch_bounds__(SCAN_THREADS) void k_mscan_sums(MultiScan<In, Out> M) {
  const int a = blockIdx.x;
  scan_tile_sums_body(M.tiles[a], M.n[a] / SCAN_TILE + 1, M.total[a]);
}

template <class In, class Out>
__global__ __launch_bounds__(SCAN_THREADS) void k_mscan_write(MultiScan<In, Out> M) {
  int64_t t;
  const int a = M.D.find(blockIdx.x, t);
  const int64_t n = M.n[a];
  const int64_t i0 = t * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  int64_t v[SCAN_ITEMS];
  mscan_load(M.in[a], i0, n, v);
  int64_t sum = 0;
#pragma unroll
  for (int j = 0; j < SCAN_ITEMS; j++) sum += v[j];
  int64_t tot;
  int64_t run = block_exclusive_scan(sum, tot) + M.tiles[a][t];
  int64_t r[SCAN_ITEMS];
#pragma unroll
  for (int j = 0; j < SCAN_ITEMS; j++) {
    r[j] = run;
    run += v[j];
  }
  mscan_store(M.out[a], i0, n, r);
}

// Sets M.D for `count` arrays (count <= MSCAN_MAX) and launches.
template <class In, class Out>
void multi_scan(MultiScan<In, Out>& M, int count, hipStream_t st) {
  M.D = depth_blocks(M.n, count, SCAN_TILE);
  const unsigned blocks = M.D.blocks();
  hipLaunchKernelGGL((k_mscan_tiles<In, Out>), dim3(blocks), dim3(SCAN_THREADS), 0, st, M);
  hipLaunchKernelGGL((k_mscan_sums<In, Out>), dim3(count), dim3(SCAN_THREADS), 0, st, M);
  hipLaunchKernelGGL((k_mscan_write<In, Out>), dim3(blocks), dim3(SCAN_THREADS), 0, st, M);
}

}  // namespace vx
