// XCD-aware work mapping.  MI355X dispatches the workgroups of a launch to its
// eight XCDs round-robin (workgroup b runs on XCD b % 8), and each XCD has its
// own L2.  Items that read the same input rows should therefore run at the
// same time on one XCD: items are dealt to the XCDs in chunks of `chunk`
// consecutive items, and the workgroups of one XCD take its chunks in order.
// Any such assignment covers every item exactly once; it only changes
// locality.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vx {

constexpr int NXCD = 8;

// Item of the u-th workgroup of XCD x: chunk u / chunk of that XCD, offset
// u % chunk.  Over u in [0, chunk * m) and x in [0, 8) this is a bijection
// onto [0, 8 * chunk * m).
__host__ __device__ inline int64_t xcd_item(int64_t x, int64_t u, int64_t chunk) {
  return ((u / chunk) * NXCD + x) * chunk + u % chunk;
}

// One item per workgroup: launch xcd_grid(items, chunk) workgroups; workgroup
// b takes item xcd_item(b % 8, b / 8, chunk) and skips it when >= items.
__host__ __device__ inline int64_t xcd_grid(int64_t items, int64_t chunk) {
  const int64_t span = NXCD * chunk;
  return (items + span - 1) / span * span;
}

// Persistent launches: workgroup b walks u = b / 8, b / 8 + (its XCD's
// workgroup count), ... (items increase with u, so the walk stops at the first
// item >= the item count).
struct XcdWalk {
  int64_t x, j, nbx, chunk;
  __device__ explicit XcdWalk(int64_t c) {
    x = blockIdx.x % NXCD;
    j = blockIdx.x / NXCD;
    nbx = ((int64_t)gridDim.x - x + NXCD - 1) / NXCD;
    chunk = c;
  }
  __device__ int64_t item(int64_t u) const { return xcd_item(x, u, chunk); }
};

}  // namespace vx
