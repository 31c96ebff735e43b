// Interval evaluation of polynomials on the boxes of one CSF level
// (Algorithm 2 of Moroz, arXiv 2406.09857, organized for gfx950).
//
// For k variables the evaluation has k stages, one per CSF depth:
//   stage 1  (depth 1, "x1 fibres"): for every depth-1 node s and every
//            trailing exponent tuple t = (e2..ek), G[s][t] = Horner over e1
//            (descending) of c[e1, t] at I1(s).  Kernel k_stage1: one lane per
//            t, R nodes of one sign class register-blocked per wave, the
//            node intervals wave-uniform.
//   stage l  (1 < l < k): for every depth-l node q under parent p and every
//            trailing tuple t of dimension k-l, Horner over e_l of
//            Cp[(e_l, t)] at I_l(q).  Kernel k_narrow: one lane per node q,
//            all lanes of a wave share the parent, so the coefficient stream
//            Cp is wave-uniform and comes in through scalar loads.
//   stage k  (leaves): E(b) = Horner over e_k of the parent's row at I_k(b),
//            then the exclusion test.  Kernel k_leaf: one lane per box.
// The chain of every (node, tuple) pair is exactly Algorithm 1 with
// consecutive exponents; chains that a wave runs together but that start
// later are fed zero coefficients first, which changes at most the sign of a
// zero (0*I + c = c).
//
// Coefficient layouts (all intervals stored as (nlo, hi) = (-lo, hi)):
//   packed (stage-1 input): rows r = 0..d for e1 = d - r; row r lists the
//     trailing tuples with |t| <= r in graded order (by |t|, then
//     lexicographic), starting at C(r+m, m+1), m = k-1.
//   O_m order (stage l input rows, stage l-1 output rows, m = k-l+1): the
//     order in which a narrow stage consumes them.  O_1 = (e = d, d-1, .., 0);
//     O_m = for t in O_{m-1}: for e = d-|t| down to 0: (e, t).  The position
//     of t in O_m is sum_{j=1..m} C(d - sigma_j + j - 1, j), sigma_j the sum
//     of t_j..t_m.
//   Rows read by the leaf kernel hold each entry as (nlo, hi, nlo), 24 bytes,
//   so that a lane can read the pair swapped by offsetting its address by 8
//   bytes (see k_leaf).
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "eval.hpp"
#include "interval.hpp"
#include "profile.hpp"
#include "scan.hpp"

namespace vx {

__host__ __device__ inline int64_t dbinom(int n, int r) {
  if (r < 0 || n < r) return 0;
  int64_t v = 1;
  for (int i = 1; i <= r; i++) v = v * (n - r + i) / i;
  return v;
}

// Rank of tuple t (dimension m <= 3) in graded order.
__device__ inline int64_t graded_rank(const int* t, int m) {
  int g = 0;
  for (int i = 0; i < m; i++) g += t[i];
  int64_t base = dbinom(g + m - 1, m);
  if (m == 2) return base + t[0];
  if (m == 3) return base + (int64_t)t[0] * (g + 1) - (int64_t)t[0] * (t[0] - 1) / 2 + t[1];
  return base;
}

// Position of tuple t (dimension m) in O_m.
__device__ inline int64_t o_pos(const int* t, int m, int d) {
  int64_t pos = 0;
  int sigma = 0;
  for (int j = m; j >= 1; j--) {
    sigma += t[j - 1];
    pos += dbinom(d - sigma + j - 1, j);
  }
  return pos;
}

// ---------------------------------------------------------------------------
// Tables and coefficient packing (one thread per cube entry).
// ---------------------------------------------------------------------------
__global__ void k_tables(int k, int d, int side, const double* __restrict__ clo, const double* __restrict__ chi,
                         double* __restrict__ packed, int2* __restrict__ ttab, int32_t* __restrict__ lens2,
                         int32_t* __restrict__ lens1) {
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t total = 1;
  for (int i = 0; i < k; i++) total *= side;
  if (f >= total) return;
  int e[VX_KMAX] = {0, 0, 0, 0};
  int64_t q = f;
  for (int i = k - 1; i >= 0; i--) { e[i] = (int)(q % side); q /= side; }
  int deg = 0;
  for (int i = 0; i < k; i++) deg += e[i];
  if (deg > d) return;
  const double lo = clo[f], hi = chi ? chi[f] : clo[f];
  const int m = k - 1;
  const int* t = e + 1;
  const int tdeg = deg - e[0];
  if (k == 1) {
    const int64_t j = d - e[0];
    packed[3 * j + 0] = -lo;
    packed[3 * j + 1] = hi;
    packed[3 * j + 2] = -lo;
    return;
  }
  const int r = d - e[0];
  const int64_t g = graded_rank(t, m);
  const int64_t at = dbinom(r + m, m + 1) + g;
  packed[2 * at + 0] = -lo;
  packed[2 * at + 1] = hi;
  if (e[0] == 0) ttab[g] = make_int2(tdeg, (int)o_pos(t, m, d));
  // chain-length tables of the narrow stages: O_2 (k = 4, stage 2) and O_1.
  if (k == 4 && e[0] == 0 && e[1] == 0) lens2[o_pos(e + 2, 2, d)] = d - (e[2] + e[3]);
  if (k >= 3) {
    bool lead_zero = true;
    for (int i = 0; i < k - 1; i++) lead_zero = lead_zero && e[i] == 0;
    if (lead_zero) lens1[d - e[k - 1]] = d - e[k - 1];
  }
}

// ---------------------------------------------------------------------------
// Work segments: runs of <= Z consecutive children of one parent that share
// a sign class.  Children are sorted by label, and the class of a cell is
// monotone in its label (NEG..., STRADDLE..., POS...), so each parent
// contributes ceil(n_neg/Z) + ceil(n_str/Z) + ceil(n_pos/Z) segments.
// ---------------------------------------------------------------------------
__device__ inline void class_bounds(const int32_t* __restrict__ labels, int64_t b, int64_t e, const AxisGrid& g,
                                    int64_t& neg_end, int64_t& pos_begin) {
  // first index whose cell has hi > 0 (end of NEG) and first with lo >= 0.
  int64_t lo = b, hi = e;
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    double nl, h;
    cell(g, labels[mid], nl, h);
    if (h <= 0.0) lo = mid + 1; else hi = mid;
  }
  neg_end = lo;
  hi = e;
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    double nl, h;
    cell(g, labels[mid], nl, h);
    if (nl <= 0.0) hi = mid; else lo = mid + 1;
  }
  pos_begin = lo;
}

__device__ inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

__global__ void k_seg_count(const int32_t* __restrict__ ptr, int64_t nparent, int64_t nchild,
                            const int32_t* __restrict__ labels, AxisGrid g, int Z, int64_t* __restrict__ cnt,
                            int64_t* __restrict__ bounds) {
  round_up_mode();
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nparent) return;
  const int64_t b = ptr ? ptr[p] : 0, e = ptr ? ptr[p + 1] : nchild;
  int64_t ne, pb;
  class_bounds(labels, b, e, g, ne, pb);
  bounds[2 * p] = ne;
  bounds[2 * p + 1] = pb;
  cnt[p] = cdiv(ne - b, Z) + cdiv(pb - ne, Z) + cdiv(e - pb, Z);
}

__global__ void k_seg_write(const int32_t* __restrict__ ptr, int64_t nparent, int64_t nchild, int Z,
                            const int64_t* __restrict__ off, const int64_t* __restrict__ bounds,
                            int4* __restrict__ seg) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nparent) return;
  const int64_t b = ptr ? ptr[p] : 0, e = ptr ? ptr[p + 1] : nchild;
  const int64_t cuts[4] = {b, bounds[2 * p], bounds[2 * p + 1], e};
  const int cls[3] = {CLS_NEG, CLS_STRADDLE, CLS_POS};
  int64_t o = off[p];
  for (int c = 0; c < 3; c++)
    for (int64_t s = cuts[c]; s < cuts[c + 1]; s += Z) {
      const int64_t cnt = cuts[c + 1] - s < Z ? cuts[c + 1] - s : Z;
      seg[o++] = make_int4((int)p, (int)s, (int)cnt, cls[c]);
    }
}

// ---------------------------------------------------------------------------
// Stage 1.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_uniform(double x) {
  const int64_t b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffff));
  const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
  return __longlong_as_double(((int64_t)hi << 32) | (uint32_t)lo);
}

template <int R, int CLS>
__device__ __forceinline__ void stage1_chain(const double2* __restrict__ P, int m, int d, int r0, int gdeg,
                                             int64_t gidx, const double (&u)[R], const double (&v)[R],
                                             const CellOps (&ops)[R], double (&nl)[R], double (&hh)[R]) {
  int64_t rowoff = dbinom(r0 + m, m + 1), rowcnt = dbinom(r0 + m, m);
  for (int r = r0; r <= d; r++) {
    double cn = 0.0, ch = 0.0;
    if (gdeg <= r) {
      const double2 c = P[rowoff + gidx];
      cn = c.x;
      ch = c.y;
    }
#pragma unroll
    for (int j = 0; j < R; j++) {
      if (CLS == CLS_POS) step_pos(nl[j], hh[j], u[j], v[j], cn, ch);
      else if (CLS == CLS_NEG) step_neg(nl[j], hh[j], u[j], v[j], cn, ch);
      else step_gen(nl[j], hh[j], ops[j], cn, ch);
    }
    rowoff += rowcnt;
    rowcnt = rowcnt * (r + m + 1) / (r + 1);
  }
}

template <int R>
__global__ __launch_bounds__(64) void k_stage1(const double2* __restrict__ P, const int2* __restrict__ ttab,
                                               int nt, int d, int m, const int32_t* __restrict__ labels0,
                                               const int4* __restrict__ seg, const int64_t* __restrict__ nseg,
                                               AxisGrid g, double* __restrict__ out, int64_t out_stride,
                                               int out_width) {
  round_up_mode();
  if ((int64_t)blockIdx.x >= *nseg) return;
  const int4 sg = seg[blockIdx.x];
  const int begin = sg.y, cnt = sg.z, cls = sg.w;
  const int lane = threadIdx.x;
  const int64_t gidx = (int64_t)blockIdx.y * 64 + lane;
  const bool active = gidx < nt;
  int gdeg = d + 1, opos = 0;
  if (active) {
    const int2 tt = ttab[gidx];
    gdeg = tt.x;
    opos = tt.y;
  }
  const int r0 = __builtin_amdgcn_readfirstlane(gdeg);  // lane 0 holds the wave's smallest |t|

  double u[R], v[R], nl[R], hh[R];
  CellOps ops[R];
#pragma unroll
  for (int j = 0; j < R; j++) {
    const int32_t lab = labels0[begin + (j < cnt ? j : 0)];
    double cnl, chi;
    cell(g, lab, cnl, chi);
    ops[j] = cell_ops(cnl, chi, cls);
    ops[j].u = wave_uniform(ops[j].u);
    ops[j].v = wave_uniform(ops[j].v);
    ops[j].nu = wave_uniform(ops[j].nu);
    ops[j].nv = wave_uniform(ops[j].nv);
    u[j] = ops[j].u;
    v[j] = ops[j].v;
    nl[j] = 0.0;
    hh[j] = 0.0;
  }
  if (cls == CLS_POS) stage1_chain<R, CLS_POS>(P, m, d, r0, gdeg, gidx, u, v, ops, nl, hh);
  else if (cls == CLS_NEG) stage1_chain<R, CLS_NEG>(P, m, d, r0, gdeg, gidx, u, v, ops, nl, hh);
  else stage1_chain<R, CLS_STRADDLE>(P, m, d, r0, gdeg, gidx, u, v, ops, nl, hh);

  if (!active) return;
#pragma unroll
  for (int j = 0; j < R; j++) {
    if (j < cnt) {
      double* o = out + (int64_t)(begin + j) * out_stride + (int64_t)opos * out_width;
      o[0] = nl[j];
      o[1] = hh[j];
      if (out_width == 3) o[2] = nl[j];
    }
  }
}

// ---------------------------------------------------------------------------
// Narrow stage.
// ---------------------------------------------------------------------------
template <int CLS>
__device__ __forceinline__ void narrow_chains(const double2* __restrict__ C, const int32_t* __restrict__ lens,
                                              int nchains, const CellOps& o, bool valid, double* __restrict__ out,
                                              int out_width) {
  int64_t pos = 0;
  for (int j = 0; j < nchains; j++) {
    const int L = lens[j];
    double2 c = C[pos];
    double nl = c.x, hh = c.y;
    for (int i = 1; i <= L; i++) {
      c = C[pos + i];
      if (CLS == CLS_POS) step_pos(nl, hh, o.u, o.v, c.x, c.y);
      else if (CLS == CLS_NEG) step_neg(nl, hh, o.u, o.v, c.x, c.y);
      else step_gen(nl, hh, o, c.x, c.y);
    }
    pos += L + 1;
    if (valid) {
      double* w = out + (int64_t)j * out_width;
      w[0] = nl;
      w[1] = hh;
      if (out_width == 3) w[2] = nl;
    }
  }
}

__global__ __launch_bounds__(64) void k_narrow(const double* __restrict__ in_rows, int64_t in_stride,
                                               const int32_t* __restrict__ lens, int nchains,
                                               const int32_t* __restrict__ labels, const int4* __restrict__ seg,
                                               const int64_t* __restrict__ nseg, AxisGrid g,
                                               double* __restrict__ out, int64_t out_stride, int out_width) {
  round_up_mode();
  if ((int64_t)blockIdx.x >= *nseg) return;
  const int4 sg = seg[blockIdx.x];
  const int parent = sg.x, begin = sg.y, cnt = sg.z, cls = sg.w;
  const int lane = threadIdx.x;
  const bool valid = lane < cnt;
  const int64_t node = begin + (valid ? lane : 0);
  double cnl, chi;
  cell(g, labels[node], cnl, chi);
  const CellOps o = cell_ops(cnl, chi, cls);
  const double2* C = reinterpret_cast<const double2*>(in_rows + (int64_t)parent * in_stride);
  double* w = out + node * out_stride;
  if (cls == CLS_POS) narrow_chains<CLS_POS>(C, lens, nchains, o, valid, w, out_width);
  else if (cls == CLS_NEG) narrow_chains<CLS_NEG>(C, lens, nchains, o, valid, w, out_width);
  else narrow_chains<CLS_STRADDLE>(C, lens, nchains, o, valid, w, out_width);
}

// ---------------------------------------------------------------------------
// Leaf stage and exclusion test.
//
// A lane whose cell is NEG evaluates the mirrored polynomial
// Ft(y) = F(-y) = sum (-1)^e c_e y^e on the nonnegative cell -I with the POS
// formula.  Negation is exact and commutes with outward rounding, so every
// intermediate value is (-1)^e times the direct one and the final value (e=0)
// is identical.  (-1)^e c_e for odd e is the pair read one double later in
// the (nlo, hi, nlo) row layout.
// ---------------------------------------------------------------------------
typedef double dpair_a8 __attribute__((ext_vector_type(2), aligned(8)));

__global__ __launch_bounds__(256) void k_leaf(const double* __restrict__ rows, int64_t row_stride,
                                              const int32_t* __restrict__ parent_of,
                                              const int32_t* __restrict__ labels, int64_t nleaf, int d,
                                              AxisGrid g, double* __restrict__ lo_out, double* __restrict__ hi_out,
                                              uint8_t* __restrict__ keep, int first) {
  round_up_mode();
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nleaf) return;
  const int64_t p = parent_of ? parent_of[b] : 0;
  double cnl, chi;
  cell(g, labels[b], cnl, chi);
  const int cls = cell_class(cnl, chi);
  const double* R = rows + p * row_stride;
  double nl, hh;
  if (cls == CLS_STRADDLE) {
    const CellOps o = cell_ops(cnl, chi, cls);
    nl = R[0];
    hh = R[1];
    for (int j = 1; j <= d; j++) step_gen(nl, hh, o, R[3 * j], R[3 * j + 1]);
  } else {
    const CellOps o = cell_ops(cnl, chi, cls);
    const int sh = cls == CLS_NEG ? 1 : 0;
    // entry j holds exponent e = d - j; mirrored lanes read odd exponents swapped.
    dpair_a8 c = *reinterpret_cast<const dpair_a8*>(R + (((d & 1) ? sh : 0)));
    nl = c.x;
    hh = c.y;
    for (int j = 1; j <= d; j++) {
      const int off = 3 * j + (((d - j) & 1) ? sh : 0);
      c = *reinterpret_cast<const dpair_a8*>(R + off);
      step_pos(nl, hh, o.u, o.v, c.x, c.y);
    }
  }
  const double lo = -opaque(nl);
  lo_out[b] = lo;
  hi_out[b] = hh;
  if (keep) {
    const bool excl = (lo > 0.0) || (hh < 0.0);
    const uint8_t kp = excl ? 0 : 1;
    keep[b] = first ? kp : (uint8_t)(keep[b] & kp);
  }
}

// Parent (depth k-1 node) of every leaf: binary search in ptr.
__global__ void k_parent_of(const int32_t* __restrict__ ptr, int64_t nparent, int64_t nleaf,
                            int32_t* __restrict__ parent) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nleaf) return;
  int64_t lo = 0, hi = nparent;  // find last p with ptr[p] <= b
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (ptr[mid] <= b) lo = mid; else hi = mid;
  }
  parent[b] = (int32_t)lo;
}

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------
struct I64Loader {
  const int64_t* a;
  __device__ int64_t operator()(int64_t i) const { return a[i]; }
};

static AxisGrid make_grid(const double* dom, int axis, int level) {
  AxisGrid g;
  g.dlo = dom[2 * axis];
  g.dhi = dom[2 * axis + 1];
  g.ndlo = -g.dlo;
  g.ndhi = -g.dhi;
  g.level = level;
  return g;
}

struct SegPlan {
  int4* seg = nullptr;
  int64_t* nseg = nullptr;
  int64_t* cnt = nullptr;
  int64_t* off = nullptr;
  int64_t* bounds = nullptr;
  int64_t* tiles = nullptr;
  int64_t nparent = 0, nchild = 0, maxseg = 0;
  int Z = 64;
};

static void plan_segments(Arena& A, SegPlan& sp, int64_t nparent, int64_t nchild, int Z) {
  sp.nparent = nparent;
  sp.nchild = nchild;
  sp.Z = Z;
  sp.maxseg = (nchild + Z - 1) / Z + 3 * nparent;
  sp.seg = A.take<int4>(sp.maxseg > 0 ? sp.maxseg : 1);
  sp.nseg = A.take<int64_t>(1);
  sp.cnt = A.take<int64_t>(nparent + 1);
  sp.off = A.take<int64_t>(nparent + 1);
  sp.bounds = A.take<int64_t>(2 * nparent + 2);
  sp.tiles = A.take<int64_t>(scan_tiles(nparent));
}

static int build_segments(SegPlan& sp, const int32_t* ptr, const int32_t* labels, const AxisGrid& g,
                          hipStream_t st) {
  const int64_t np = sp.nparent;
  if (np == 0) {
    VX_HIP(hipMemsetAsync(sp.nseg, 0, sizeof(int64_t), st));
    return VX_OK;
  }
  const unsigned blocks = (unsigned)((np + 255) / 256);
  hipLaunchKernelGGL(k_seg_count, dim3(blocks), dim3(256), 0, st, ptr, np, sp.nchild, labels, g, sp.Z, sp.cnt,
                     sp.bounds);
  VX_CHECK_LAUNCH("k_seg_count");
  scan_exclusive(I64Loader{sp.cnt}, (const int64_t*)nullptr, np, sp.off, sp.nseg, sp.tiles, st);
  VX_CHECK_LAUNCH("segment scan");
  hipLaunchKernelGGL(k_seg_write, dim3(blocks), dim3(256), 0, st, ptr, np, sp.nchild, sp.Z,
                     (const int64_t*)sp.off, (const int64_t*)sp.bounds, sp.seg);
  VX_CHECK_LAUNCH("k_seg_write");
  return VX_OK;
}

constexpr int STAGE1_R = 8;

struct EvalPlan {
  int k = 0, dmax = 0;
  double* packed = nullptr;
  int2* ttab = nullptr;
  int32_t* lens2 = nullptr;
  int32_t* lens1 = nullptr;
  double* rows[VX_KMAX] = {nullptr, nullptr, nullptr, nullptr};  // output rows of stage l (l = 0..k-2)
  int32_t* parent = nullptr;
  SegPlan seg[VX_KMAX];
};

// Workspace layout of one interval_eval_level call (measure with A.base == nullptr).
static void plan_eval(Arena& A, EvalPlan& E, const vx_poly* P, int np, const vx_csf* S) {
  const int k = S->k;
  int dmax = 0;
  for (int p = 0; p < np; p++) dmax = P[p].degree > dmax ? P[p].degree : dmax;
  E.k = k;
  E.dmax = dmax;
  const int64_t nt_k = ntup(k, dmax);
  E.packed = A.take<double>(k == 1 ? 3 * (int64_t)(dmax + 1) : 2 * nt_k);
  E.ttab = A.take<int2>(k >= 2 ? ntup(k - 1, dmax) : 1);
  E.lens2 = A.take<int32_t>(k == 4 ? ntup(2, dmax) : 1);
  E.lens1 = A.take<int32_t>(dmax + 1);
  for (int l = 0; l + 1 < k; l++) {
    const int m = k - l - 1;  // dimension of the trailing tuples left after depth l+1
    const int width = (l == k - 2) ? 3 : 2;
    E.rows[l] = A.take<double>((size_t)S->n[l] * ntup(m, dmax) * width);
  }
  if (k >= 2) E.parent = A.take<int32_t>(S->n[k - 1] > 0 ? S->n[k - 1] : 1);
  for (int l = 0; l + 1 < k; l++) {
    const int64_t nparent = l == 0 ? 1 : S->n[l - 1];
    plan_segments(A, E.seg[l], nparent, S->n[l], l == 0 ? STAGE1_R : 64);
  }
}

size_t eval_workspace_bytes(const vx_poly* P, int np, const vx_csf* S) {
  Arena A;
  EvalPlan E;
  plan_eval(A, E, P, np, S);
  return A.off + 256;
}

int eval_level_impl(const vx_poly* P, int np, const vx_csf* S, const double* dom, double* lo, double* hi,
                    uint8_t* keep, void* ws, size_t ws_bytes, hipStream_t st) {
  const int k = S->k;
  const int64_t nleaf = S->n[k - 1];
  if (nleaf == 0) return VX_OK;
  Arena A;
  A.base = reinterpret_cast<char*>(ws);
  A.size = ws_bytes;
  EvalPlan E;
  plan_eval(A, E, P, np, S);
  if (A.overflow)
    VX_FAIL(VX_ECAPACITY, "interval_eval_level: workspace of %zu bytes is too small (%zu needed)", ws_bytes,
            A.off + 256);

  // Segments (depend on the CSF only).
  for (int l = 0; l + 1 < k; l++) {
    const AxisGrid g = make_grid(dom, l, S->level);
    int rc = build_segments(E.seg[l], l == 0 ? nullptr : S->ptr[l - 1], S->idx[l], g, st);
    if (rc) return rc;
  }
  if (k >= 2) {
    hipLaunchKernelGGL(k_parent_of, dim3((unsigned)((nleaf + 255) / 256)), dim3(256), 0, st, S->ptr[k - 2],
                       S->n[k - 2], nleaf, E.parent);
    VX_CHECK_LAUNCH("k_parent_of");
  }
  const AxisGrid gleaf = make_grid(dom, k - 1, S->level);

  for (int p = 0; p < np; p++) {
    const int d = P[p].degree, side = P[p].side;
    int64_t cube = 1;
    for (int i = 0; i < k; i++) cube *= side;
    hipLaunchKernelGGL(k_tables, dim3((unsigned)((cube + 255) / 256)), dim3(256), 0, st, k, d, side, P[p].c_lo,
                       P[p].c_hi, E.packed, E.ttab, E.lens2, E.lens1);
    VX_CHECK_LAUNCH("k_tables");
    if (k == 1) {
      const int ps = prof_start("k_leaf", (double)d * (double)nleaf, st);
      hipLaunchKernelGGL(k_leaf, dim3((unsigned)((nleaf + 255) / 256)), dim3(256), 0, st, (const double*)E.packed,
                         (int64_t)0, (const int32_t*)nullptr, S->idx[0], nleaf, d, gleaf, lo + p * nleaf,
                         hi + p * nleaf, keep, p == 0 ? 1 : 0);
      VX_CHECK_LAUNCH("k_leaf");
      prof_stop(ps, st);
      continue;
    }
    // stage 1
    {
      const int m = k - 1;
      const int64_t nt = ntup(m, d);
      const int width = (k == 2) ? 3 : 2;
      const int64_t stride = nt * width;
      const SegPlan& sp = E.seg[0];
      dim3 grid((unsigned)sp.maxseg, (unsigned)((nt + 63) / 64));
      const int ps = prof_start("k_stage1", (double)(ntup(k, d) - nt) * (double)S->n[0], st);
      hipLaunchKernelGGL(k_stage1<STAGE1_R>, grid, dim3(64), 0, st, (const double2*)E.packed,
                         (const int2*)E.ttab, (int)nt, d, m, S->idx[0], (const int4*)sp.seg,
                         (const int64_t*)sp.nseg, make_grid(dom, 0, S->level), E.rows[0], stride, width);
      VX_CHECK_LAUNCH("k_stage1");
      prof_stop(ps, st);
    }
    // middle stages
    for (int l = 1; l + 1 < k; l++) {
      const int m_in = k - l;        // tuple dimension of the parent rows
      const int m_out = k - l - 1;   // chains of this stage
      const int64_t nch = ntup(m_out, d);
      const int width = (l == k - 2) ? 3 : 2;
      const SegPlan& sp = E.seg[l];
      const int32_t* lens = (m_out == 2) ? E.lens2 : E.lens1;
      const int ps = prof_start("k_narrow", (double)(ntup(m_in, d) - nch) * (double)S->n[l], st);
      hipLaunchKernelGGL(k_narrow, dim3((unsigned)sp.maxseg), dim3(64), 0, st, (const double*)E.rows[l - 1],
                         (int64_t)(ntup(m_in, d) * 2), lens, (int)nch, S->idx[l], (const int4*)sp.seg,
                         (const int64_t*)sp.nseg, make_grid(dom, l, S->level), E.rows[l], nch * width, width);
      VX_CHECK_LAUNCH("k_narrow");
      prof_stop(ps, st);
    }
    // leaves
    const int ps = prof_start("k_leaf", (double)d * (double)nleaf, st);
    hipLaunchKernelGGL(k_leaf, dim3((unsigned)((nleaf + 255) / 256)), dim3(256), 0, st,
                       (const double*)E.rows[k - 2], (int64_t)(3 * (d + 1)), (const int32_t*)E.parent,
                       S->idx[k - 1], nleaf, d, gleaf, lo + p * nleaf, hi + p * nleaf, keep, p == 0 ? 1 : 0);
    VX_CHECK_LAUNCH("k_leaf");
    prof_stop(ps, st);
  }
  return VX_OK;
}

}  // namespace vx
