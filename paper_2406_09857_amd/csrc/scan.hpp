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

// Exclusive scan of one value per thread across the workgroup; returns the
// thread's exclusive prefix and writes the workgroup total to `total`.
__device__ __forceinline__ int64_t block_exclusive_scan(int64_t v, int64_t& total) {
  __shared__ int64_t wsum[SCAN_THREADS / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int64_t inc = wave_inclusive_scan(v);
  if (lane == 63) wsum[wid] = inc;
  __syncthreads();
  int64_t base = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < SCAN_THREADS / 64; w++) {
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

// Several independent exclusive scans in three launches, blockIdx.y picking
// the array: out_a[0..n_a] = exclusive prefix sums of in_a, out_a[n_a] =
// total_a = *total[a].  Inputs are 0/1 flags (uint8, nonzero counts as 1) or
// int64 counts; tiles[a] needs scan_tiles(n_a) int64s.
constexpr int MSCAN_MAX = 4;

__device__ __forceinline__ int64_t mscan_value(uint8_t v) { return v != 0; }
__device__ __forceinline__ int64_t mscan_value(int64_t v) { return v; }

template <class In, class Out>
struct MultiScan {
  const In* in[MSCAN_MAX];
  Out* out[MSCAN_MAX];
  int64_t* total[MSCAN_MAX];
  int64_t* tiles[MSCAN_MAX];
  int64_t n[MSCAN_MAX];
};

template <class In, class Out>
__global__ __launch_bounds__(SCAN_THREADS) void k_mscan_tiles(MultiScan<In, Out> M) {
  const int a = blockIdx.y;
  const int64_t n = M.n[a];
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
  if (base > n) return;  // tiles 0 .. n / SCAN_TILE exist for every array
  const int64_t i0 = base + (int64_t)threadIdx.x * SCAN_ITEMS;
  int64_t sum = 0;
#pragma unroll
  for (int j = 0; j < SCAN_ITEMS; j++)
    if (i0 + j < n) sum += mscan_value(M.in[a][i0 + j]);
  int64_t tot;
  block_exclusive_scan(sum, tot);
  if (threadIdx.x == 0) M.tiles[a][blockIdx.x] = tot;
}

template <class In, class Out>
__global__ __launch_bounds__(SCAN_THREADS) void k_mscan_sums(MultiScan<In, Out> M) {
  const int a = blockIdx.y;
  scan_tile_sums_body(M.tiles[a], M.n[a] / SCAN_TILE + 1, M.total[a]);
}

template <class In, class Out>
__global__ __launch_bounds__(SCAN_THREADS) void k_mscan_write(MultiScan<In, Out> M) {
  const int a = blockIdx.y;
  const int64_t n = M.n[a];
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
  if (base > n) return;
  const int64_t i0 = base + (int64_t)threadIdx.x * SCAN_ITEMS;
  int64_t v[SCAN_ITEMS];
  int64_t sum = 0;
#pragma unroll
  for (int j = 0; j < SCAN_ITEMS; j++) {
    v[j] = i0 + j < n ? mscan_value(M.in[a][i0 + j]) : 0;
    sum += v[j];
  }
  int64_t tot;
  int64_t run = block_exclusive_scan(sum, tot) + M.tiles[a][blockIdx.x];
#pragma unroll
  for (int j = 0; j < SCAN_ITEMS; j++) {
    if (i0 + j <= n) M.out[a][i0 + j] = (Out)run;
    run += v[j];
  }
}

// count arrays (count <= MSCAN_MAX), nmax = the largest n.
template <class In, class Out>
void multi_scan(const MultiScan<In, Out>& M, int count, int64_t nmax, hipStream_t st) {
  const dim3 grid((unsigned)(nmax / SCAN_TILE + 1), (unsigned)count);
  hipLaunchKernelGGL((k_mscan_tiles<In, Out>), grid, dim3(SCAN_THREADS), 0, st, M);
  hipLaunchKernelGGL((k_mscan_sums<In, Out>), dim3(1, count), dim3(SCAN_THREADS), 0, st, M);
  hipLaunchKernelGGL((k_mscan_write<In, Out>), grid, dim3(SCAN_THREADS), 0, st, M);
}

}  // namespace vx
