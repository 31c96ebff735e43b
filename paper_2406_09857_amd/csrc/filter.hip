// Exclusion filter, bisection and CSF compaction (Algorithm 3 of Moroz,
// arXiv 2406.09857; bisection of G_n into G_2n, Sec. 3.2).
//
// Given a level's CSF S and a keep flag per box:
//   K    = S restricted to the kept boxes; an internal node survives when at
//          least one descendant box does.  Depth by depth from the leaves:
//          newpos_l = exclusive scan of the survival flags, and a node's flag
//          is newpos_{l+1}[ptr[q+1]] > newpos_{l+1}[ptr[q]].
//   next = CSF of the children 2B + c, c in {0,1}^k, of every kept box B.  A
//          depth-l node z of K with label i (ancestors a_0 .. a_l = z) becomes
//          the 2^(l+1) nodes (bits b_0 .. b_l) with labels 2 i + b_l, so
//          N_l(next) = 2^(l+1) N_l(K).  Next's nodes are ordered by
//          (a_0, b_0, a_1, b_1, ...), so with F_l(x) = index of the first
//          depth-l descendant in K of node x (at depth i: kptr chained l - i
//          times) the position of the copy is
//            sum_i 2^(l-i+1) (F_l(a_i) - F_l(a_(i-1))) + b_i 2^(l-i) (F_l(a_i + 1) - F_l(a_i)),
//          F_l(a_(-1)) = 0, and its child offset is the position of the copy
//          (b_0 .. b_l, 0) of z's first kept child.  Every node of next is
//          written by the thread of its K node, without scans or searches.
// Large levels take seven launches: survival flags of the inner depths
// (leaves up), one multi-array scan of every depth's flags, compaction of
// every depth (which also records each kept node's parent), and the next CSF.
// All passes have one thread per element and no atomics; nothing depends on
// scheduling order, so the output is deterministic.
#include <hip/hip_runtime.h>
#include <string.h>

#include "common.hpp"
#include "eval.hpp"
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

static_assert(MSCAN_MAX >= VX_KMAX, "one scan array per depth");

// Publish the counts: *flag = value once the counts written before by this
// thread are visible to the host.
__device__ __forceinline__ void publish_counts(int64_t* flag, int64_t value) {
  if (!flag) return;
  __threadfence_system();
  *reinterpret_cast<volatile int64_t*>(flag) = value;
}


// Survival flag of every depth-l node (l < k-1): some child survives.  One
// thread per node reads its children's flags eight bytes at a time, eight
// words in flight, and stops at the first batch holding a survivor.  Bytes of
// a word outside the node's range are masked; the word holding the array's
// last byte, and every word of a flag array that is not 8-byte aligned, are
// read bytewise so that nothing past the array is touched.
constexpr int ALIVE_BATCH = 8;

__device__ __forceinline__ uint64_t flag_word(const uint8_t* __restrict__ f, int64_t wi, int64_t nf, bool aligned) {
  if (aligned && (wi + 1) * 8 <= nf) return reinterpret_cast<const uint64_t*>(f)[wi];
  uint64_t v = 0;
  for (int j = 0; j < 8; j++) {
    const int64_t c = wi * 8 + j;
    if (c >= 0 && c < nf) v |= (uint64_t)f[c] << (8 * j);
  }
  return v;
}

__global__ void k_alive(int64_t n, const int32_t* __restrict__ ptr, const uint8_t* __restrict__ child_alive,
                        int64_t nchild, uint8_t* __restrict__ alive) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const bool aligned = ((uintptr_t)child_alive & 7) == 0;
  const int64_t b = ptr[p], e = ptr[p + 1];
  const int64_t we = (e + 7) >> 3;  // one past the last word
  bool a = false;
  for (int64_t wb = b >> 3; wb < we && !a; wb += ALIVE_BATCH) {
    uint64_t acc = 0;
#pragma unroll
    for (int u = 0; u < ALIVE_BATCH; u++) {
      const int64_t wi = wb + u;
      if (wi < we) {
        uint64_t v = flag_word(child_alive, wi, nchild, aligned);
        const int64_t lo = b - wi * 8, hi = e - wi * 8;  // the node's bytes within this word
        if (lo > 0) v &= ~0ull << (8 * lo);
        if (hi < 8) v &= ~0ull >> (8 * (8 - hi));
        acc |= v;
      }
    }
    a = acc != 0;
  }
  alive[p] = a;
}

struct CompactJob {
  const int32_t* idx[VX_KMAX];
  const int32_t* ptr[VX_KMAX];
  const int32_t* newpos[VX_KMAX];
  int32_t* kidx[VX_KMAX];
  int32_t* kptr[VX_KMAX];
  int32_t* kpar[VX_KMAX];  // kpar[l][j] = parent (depth l-1 index in K) of kept node j; null: not wanted
  int64_t n[VX_KMAX];
  const int64_t* kcnt;
  int64_t* ncnt;
  int64_t* d_counts;
  int64_t* flag;
  int64_t flag_value;
};

// Kept nodes of every depth (one 1-D grid over the depths).  A surviving
// node p lands at newpos[p]; its kept children are the contiguous range
// newpos'[ptr[p]] .. newpos'[ptr[p+1]] of the next depth.
__global__ void k_compact_all(int k, DepthBlocks D, CompactJob J) {
  int64_t t;
  const int l = D.find(blockIdx.x, t);
  const bool inner = l + 1 < k;
  if (t == 0 && threadIdx.x == 0) {
    if (inner) J.kptr[l][J.kcnt[l]] = (int32_t)J.kcnt[l + 1];
    if (l == 0) {
      for (int m = 0; m < k; m++) {
        J.ncnt[m] = J.kcnt[m] << (m + 1);
        if (J.d_counts) {
          J.d_counts[m] = J.kcnt[m];
          J.d_counts[k + m] = J.ncnt[m];
        }
      }
      publish_counts(J.flag, J.flag_value);
    }
  }
  const int64_t p = t * blockDim.x + threadIdx.x;
  if (p >= J.n[l]) return;
  const int32_t q = J.newpos[l][p];
  if (J.newpos[l][p + 1] == q) return;
  J.kidx[l][q] = J.idx[l][p];
  if (inner) {
    const int32_t c0 = J.newpos[l + 1][J.ptr[l][p]], c1 = J.newpos[l + 1][J.ptr[l][p + 1]];
    J.kptr[l][q] = c0;
    if (J.kpar[l + 1])
      for (int32_t c = c0; c < c1; c++) J.kpar[l + 1][c] = q;
  }
}

struct GenJob {
  const int32_t* kidx[VX_KMAX];
  const int32_t* kptr[VX_KMAX];
  const int32_t* kpar[VX_KMAX];
  int32_t* nidx[VX_KMAX];
  int32_t* nptr[VX_KMAX];
  const int64_t* kcnt;
  const int64_t* ncnt;
};

// Index of the first depth-L descendant in K of the depth-i node x (x may be
// one past the last node of its depth).
template <int L>
__device__ __forceinline__ int64_t first_desc(const GenJob& J, int i, int64_t x) {
#pragma unroll
  for (int m = 0; m < L; m++)
    if (m >= i) x = J.kptr[m][x];
  return x;
}

// Position terms of the copies at depth L of the node with ancestors a[0..L]:
// position(bits) = base + sum over set bits i of w[i] (bit i = b_i).
template <int L>
__device__ __forceinline__ void copy_terms(const GenJob& J, const int64_t* a, int64_t& base, int64_t* w) {
  base = 0;
  int64_t prev = 0;
#pragma unroll
  for (int i = 0; i <= L; i++) {
    const int64_t f0 = first_desc<L>(J, i, a[i]);
    const int64_t f1 = first_desc<L>(J, i, a[i] + 1);
    base += (f0 - prev) << (L - i + 1);
    w[i] = (f1 - f0) << (L - i);
    prev = f0;
  }
}

// The 2^(L+1) copies in next of kept depth-L node z, with their labels and
// (inner depths) child offsets.
template <int L>
__device__ __forceinline__ void next_copies(const GenJob& J, int64_t z, bool inner) {
  int64_t a[L + 2];
  a[L] = z;
#pragma unroll
  for (int i = L; i > 0; i--) a[i - 1] = J.kpar[i][a[i]];
  int64_t base, w[L + 1];
  copy_terms<L>(J, a, base, w);
  int64_t cbase = 0, cw[L + 2];
  if (inner) {
    a[L + 1] = J.kptr[L][z];
    copy_terms<L + 1>(J, a, cbase, cw);
  }
  const int32_t lab = 2 * J.kidx[L][z];
  for (unsigned hi = 0; hi < (1u << L); hi++) {  // b_0 .. b_(L-1)
    int64_t o = base, c = cbase;
#pragma unroll
    for (int i = 0; i < L; i++)
      if ((hi >> i) & 1) {
        o += w[i];
        c += inner ? cw[i] : 0;
      }
#pragma unroll
    for (int b = 0; b < 2; b++) {  // b_L
      const int64_t ob = o + (b ? w[L] : 0);
      J.nidx[L][ob] = lab + b;
      if (inner) J.nptr[L][ob] = (int32_t)(c + (b ? cw[L] : 0));
    }
  }
}

// Next CSF, every depth (one 1-D grid over the depths), one thread per kept node.
__global__ void k_next_gen(int k, DepthBlocks D, GenJob J) {
  int64_t t;
  const int l = D.find(blockIdx.x, t);
  const bool inner = l + 1 < k;
  if (t == 0 && threadIdx.x == 0 && inner) J.nptr[l][J.ncnt[l]] = (int32_t)J.ncnt[l + 1];
  const int64_t z = t * blockDim.x + threadIdx.x;
  if (z >= J.kcnt[l]) return;
  switch (l) {
    case 0: next_copies<0>(J, z, inner); break;
    case 1: next_copies<1>(J, z, inner); break;
    case 2: next_copies<2>(J, z, inner); break;
    default: next_copies<3>(J, z, inner); break;
  }
}

// ---------------------------------------------------------------------------
// Small levels: the whole filter in one workgroup of SMALL_FILTER_THREADS
// (survival scans leaves up, compaction of every depth in one pass with the
// kept nodes' parents, the next CSF of every depth in one pass in closed
// form), the same outputs as the multi-launch path.
// ---------------------------------------------------------------------------
constexpr int64_t SMALL_FILTER_NODES = 1024;
constexpr int SMALL_FILTER_THREADS = 1024;

struct SmallFilterJob {
  const int32_t* idx[VX_KMAX];
  const int32_t* ptr[VX_KMAX];
  int64_t n[VX_KMAX];
  int32_t* newpos[VX_KMAX];
  int32_t* kidx[VX_KMAX];
  int32_t* kptr[VX_KMAX];
  int32_t* kpar[VX_KMAX];
  int32_t* nidx[VX_KMAX];
  int32_t* nptr[VX_KMAX];
  int64_t* kcnt;
  int64_t* ncnt;
  int64_t* d_counts;
  int64_t* flag;
  int64_t flag_value;
};

// out[0..n] = exclusive prefix sums of ld(0..n-1); returns the total (all threads).
template <class Loader>
__device__ int64_t block_scan_to(Loader ld, int64_t n, int32_t* out) {
  constexpr int64_t TILE = (int64_t)SMALL_FILTER_THREADS * SCAN_ITEMS;
  int64_t carry = 0;
  for (int64_t base = 0; base < n; base += TILE) {
    const int64_t i0 = base + (int64_t)threadIdx.x * SCAN_ITEMS;
    int64_t v[SCAN_ITEMS];
    int64_t sum = 0;
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; j++) {
      v[j] = i0 + j < n ? ld(i0 + j) : 0;
      sum += v[j];
    }
    int64_t tot;
    int64_t run = carry + block_exclusive_scan<SMALL_FILTER_THREADS>(sum, tot);
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

__global__ __launch_bounds__(SMALL_FILTER_THREADS) void k_filter_small(int k, const uint8_t* __restrict__ keep,
                                                                       SmallFilterJob J, int want_next) {
  int64_t kc[VX_KMAX] = {0, 0, 0, 0};
  kc[k - 1] = block_scan_to(KeepLoader{keep}, J.n[k - 1], J.newpos[k - 1]);
  for (int l = k - 2; l >= 0; l--)
    kc[l] = block_scan_to(AnyChildLoader{J.ptr[l], J.newpos[l + 1]}, J.n[l], J.newpos[l]);
  // the counts are final: publish them before the compaction and the next CSF
  if (threadIdx.x == 0) {
    for (int l = 0; l < k; l++) {
      if (l + 1 < k) J.kptr[l][kc[l]] = (int32_t)kc[l + 1];
      J.kcnt[l] = kc[l];
      J.ncnt[l] = kc[l] << (l + 1);
      if (J.d_counts) {
        J.d_counts[l] = kc[l];
        J.d_counts[k + l] = kc[l] << (l + 1);
      }
      if (want_next && l + 1 < k) J.nptr[l][kc[l] << (l + 1)] = (int32_t)(kc[l + 1] << (l + 2));
    }
    publish_counts(J.flag, J.flag_value);
  }
  int64_t items = 0;
  for (int l = 0; l < k; l++) items += J.n[l];
  for (int64_t i = threadIdx.x; i < items; i += SMALL_FILTER_THREADS) {
    int64_t p = i;
    int l = 0;
    while (l + 1 < k && p >= J.n[l]) p -= J.n[l++];
    const int32_t q = J.newpos[l][p];
    if (J.newpos[l][p + 1] == q) continue;
    J.kidx[l][q] = J.idx[l][p];
    if (l + 1 < k) {
      const int32_t c0 = J.newpos[l + 1][J.ptr[l][p]], c1 = J.newpos[l + 1][J.ptr[l][p + 1]];
      J.kptr[l][q] = c0;
      if (want_next)
        for (int32_t c = c0; c < c1; c++) J.kpar[l + 1][c] = q;
    }
  }
  if (!want_next) return;
  __syncthreads();
  GenJob G;
  for (int l = 0; l < VX_KMAX; l++) {
    G.kidx[l] = J.kidx[l];
    G.kptr[l] = J.kptr[l];
    G.kpar[l] = J.kpar[l];
    G.nidx[l] = J.nidx[l];
    G.nptr[l] = J.nptr[l];
  }
  G.kcnt = J.kcnt;
  G.ncnt = J.ncnt;
  int64_t kitems = 0;
  for (int l = 0; l < k; l++) kitems += kc[l];
  for (int64_t i = threadIdx.x; i < kitems; i += SMALL_FILTER_THREADS) {
    int64_t z = i;
    int l = 0;
    while (l + 1 < k && z >= kc[l]) z -= kc[l++];
    const bool inner = l + 1 < k;
    switch (l) {
      case 0: next_copies<0>(G, z, inner); break;
      case 1: next_copies<1>(G, z, inner); break;
      case 2: next_copies<2>(G, z, inner); break;
      default: next_copies<3>(G, z, inner); break;
    }
  }
}

struct FilterPlan {
  int32_t* newpos[VX_KMAX] = {};
  uint8_t* alive[VX_KMAX] = {};
  int64_t* kcnt = nullptr;
  int64_t* ncnt = nullptr;
  int64_t* tiles[VX_KMAX] = {};
  int32_t* kidx[VX_KMAX] = {};
  int32_t* kptr[VX_KMAX] = {};
  int32_t* kpar[VX_KMAX] = {};
};

static void plan_filter(Arena& A, FilterPlan& F, const vx_csf* S, bool own_kept, bool want_next) {
  const int k = S->k;
  for (int l = 0; l < k; l++) {
    F.newpos[l] = A.take<int32_t>(S->n[l] + 1);
    F.tiles[l] = A.take<int64_t>(scan_tiles(S->n[l]));
    if (l + 1 < k) F.alive[l] = A.take<uint8_t>(S->n[l] > 0 ? S->n[l] : 1);
  }
  F.kcnt = A.take<int64_t>(VX_KMAX);
  F.ncnt = A.take<int64_t>(VX_KMAX);
  if (own_kept)
    for (int l = 0; l < k; l++) {
      F.kidx[l] = A.take<int32_t>(S->n[l] > 0 ? S->n[l] : 1);
      if (l + 1 < k) F.kptr[l] = A.take<int32_t>(S->n[l] + 1);
    }
  if (want_next)
    for (int l = 1; l < k; l++) F.kpar[l] = A.take<int32_t>(S->n[l] > 0 ? S->n[l] : 1);
}

size_t filter_workspace_bytes(const vx_csf* S) {
  Arena A;
  FilterPlan F;
  plan_filter(A, F, S, true, true);
  return A.off + 256;
}

static int filter_body(const vx_csf* S, const uint8_t* keep, vx_csf* kept, vx_csf* next, int64_t* d_counts,
                       void* ws, size_t ws_bytes, hipStream_t st, int64_t* flag, int64_t flag_value,
                       const uint8_t* alive_km2);

int filter_impl(const vx_csf* S, const uint8_t* keep, vx_csf* kept, vx_csf* next, int64_t* d_counts, void* ws,
                size_t ws_bytes, hipStream_t st, int64_t* flag, int64_t flag_value, const uint8_t* alive) {
  const int ps = prof_start("filter_subdivide", (double)S->n[S->k - 1], st);
  const int rc = filter_body(S, keep, kept, next, d_counts, ws, ws_bytes, st, flag, flag_value, alive);
  prof_stop(ps, st);
  return rc;
}

static int filter_body(const vx_csf* S, const uint8_t* keep, vx_csf* kept, vx_csf* next, int64_t* d_counts,
                       void* ws, size_t ws_bytes, hipStream_t st, int64_t* flag, int64_t flag_value,
                       const uint8_t* alive_km2) {
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
      J.kpar[l] = F.kpar[l];
    }
    J.kcnt = F.kcnt;
    J.ncnt = F.ncnt;
    J.d_counts = d_counts;
    J.flag = flag;
    J.flag_value = flag_value;
    hipLaunchKernelGGL(k_filter_small, dim3(1), dim3(SMALL_FILTER_THREADS), 0, st, k, keep, J, next ? 1 : 0);
    VX_CHECK_LAUNCH("k_filter_small");
    return VX_OK;
  }

  // Survival flags of the inner depths, leaves up (depth k-2 possibly given);
  // then every depth's scan.
  for (int l = k - 2; l >= 0; l--) {
    if (l == k - 2 && alive_km2) {
      F.alive[l] = const_cast<uint8_t*>(alive_km2);
      continue;
    }
    const int64_t n = S->n[l];
    hipLaunchKernelGGL(k_alive, dim3((unsigned)((n + 255) / 256 > 0 ? (n + 255) / 256 : 1)), dim3(256), 0, st, n,
                       (const int32_t*)S->ptr[l], l + 2 < k ? (const uint8_t*)F.alive[l + 1] : keep, S->n[l + 1],
                       F.alive[l]);
    VX_CHECK_LAUNCH("k_alive");
  }
  MultiScan<uint8_t, int32_t> M;
  memset(&M, 0, sizeof M);
  for (int l = 0; l < k; l++) {
    M.in[l] = l + 1 < k ? F.alive[l] : keep;
    M.out[l] = F.newpos[l];
    M.total[l] = F.kcnt + l;
    M.tiles[l] = F.tiles[l];
    M.n[l] = S->n[l];
  }
  multi_scan(M, k, st);
  VX_CHECK_LAUNCH("survival scans");
  // Compacted K (and each kept node's parent when next is wanted).
  CompactJob C;
  memset(&C, 0, sizeof C);
  for (int l = 0; l < k; l++) {
    C.idx[l] = S->idx[l];
    C.ptr[l] = l + 1 < k ? S->ptr[l] : nullptr;
    C.newpos[l] = F.newpos[l];
    C.kidx[l] = kidx[l];
    C.kptr[l] = l + 1 < k ? kptr[l] : nullptr;
    C.kpar[l] = next ? F.kpar[l] : nullptr;
    C.n[l] = S->n[l];
  }
  C.kcnt = F.kcnt;
  C.ncnt = F.ncnt;
  C.d_counts = d_counts;
  C.flag = flag;
  C.flag_value = flag_value;
  const DepthBlocks D = depth_blocks(S->n, k, 256);
  hipLaunchKernelGGL(k_compact_all, dim3(D.blocks()), dim3(256), 0, st, k, D, C);
  VX_CHECK_LAUNCH("k_compact_all");
  if (!next) return VX_OK;
  // Children CSF.
  GenJob G;
  memset(&G, 0, sizeof G);
  for (int l = 0; l < k; l++) {
    G.kidx[l] = kidx[l];
    G.kptr[l] = l + 1 < k ? kptr[l] : nullptr;
    G.kpar[l] = F.kpar[l];
    G.nidx[l] = next->idx[l];
    G.nptr[l] = l + 1 < k ? next->ptr[l] : nullptr;
  }
  G.kcnt = F.kcnt;
  G.ncnt = F.ncnt;
  hipLaunchKernelGGL(k_next_gen, dim3(D.blocks()), dim3(256), 0, st, k, D, G);
  VX_CHECK_LAUNCH("k_next_gen");
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
