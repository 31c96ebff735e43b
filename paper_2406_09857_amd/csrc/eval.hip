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
//   Rows read by the leaf kernel hold each entry as the pair (nlo, hi), 16
//   bytes (LEAF_W doubles); a lane that needs the pair swapped loads the two
//   doubles from swapped offsets (see leaf_chains).
#include <hip/hip_runtime.h>

#include <string.h>

#include <vector>

#include "common.hpp"
#include "eval.hpp"
#include "fill.hpp"
#include "interval.hpp"
#include "profile.hpp"
#include "scan.hpp"
#include "xcd.hpp"

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

// Padded O_2 layout (k = 3, input rows of the middle stage): chain j of O_1
// (exponent e3 = d - j, j+1 entries) is preceded by zero entries up to a
// multiple of 8 entries, so it occupies the 8-entry groups [c(j), c(j+1)),
// c(j) = sum_{i=1..j} ceil(i/8).  Entry (e2, e3) sits at 8 c(j+1) - 1 - e2.
constexpr int PADG = 8;
// Doubles per entry of the leaf kernel's input rows: (nlo, hi).
constexpr int LEAF_W = 2;
constexpr int SEG_PACKED = 4;  // segment class | this flag: a packed middle-stage segment

__host__ __device__ inline int64_t padded_groups(int64_t j) {
  const int64_t q = j / PADG, r = j % PADG;
  return (PADG / 2) * q * (q + 1) + (q + 1) * r;
}

__host__ __device__ inline int64_t padded_entries(int d) { return PADG * padded_groups(d + 1); }

__host__ __device__ inline int64_t padded_npad(int d) {
  return padded_entries(d) - (int64_t)(d + 1) * (d + 2) / 2;
}

// ---------------------------------------------------------------------------
// Tables and coefficient packing (one thread per cube entry).
// ---------------------------------------------------------------------------
__device__ inline void tables_entry(int64_t f, int k, int d, int side, const double* __restrict__ clo,
                                    const double* __restrict__ chi, double* __restrict__ packed,
                                    int2* __restrict__ ttab, int32_t* __restrict__ lens2,
                                    int32_t* __restrict__ lens1, int32_t* __restrict__ padlist) {
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
  if (f == 0 && k >= 2) {  // zero entry after the last row (read by chains not yet started)
    packed[2 * dbinom(d + k, k) + 0] = 0.0;
    packed[2 * dbinom(d + k, k) + 1] = 0.0;
  }
  if (k == 1) {
    const int64_t j = d - e[0];
    packed[LEAF_W * j + 0] = -lo;
    packed[LEAF_W * j + 1] = hi;
    return;
  }
  const int r = d - e[0];
  const int64_t g = graded_rank(t, m);
  const int64_t at = dbinom(r + m, m + 1) + g;
  packed[2 * at + 0] = -lo;
  packed[2 * at + 1] = hi;
  if (e[0] == 0) {
    if (k == 3) {
      const int j = d - e[2];
      ttab[g] = make_int2(tdeg, (int)(PADG * padded_groups(j + 1) - 1 - e[1]));
      if (e[1] == 0) {  // one thread per chain lists the chain's padding slots
        const int64_t start = PADG * padded_groups(j);
        const int64_t pad = PADG * padded_groups(j + 1) - start - (j + 1);
        const int64_t at0 = start - (int64_t)j * (j + 1) / 2;
        for (int64_t q2 = 0; q2 < pad; q2++) padlist[at0 + q2] = (int32_t)(start + q2);
      }
    } else {
      ttab[g] = make_int2(tdeg, (int)o_pos(t, m, d));
    }
  }
  // chain-length tables of the narrow stages: O_2 (k = 4, stage 2) and O_1.
  if (k == 4 && e[0] == 0 && e[1] == 0) lens2[o_pos(e + 2, 2, d)] = d - (e[2] + e[3]);
  if (k >= 3) {
    bool lead_zero = true;
    for (int i = 0; i < k - 1; i++) lead_zero = lead_zero && e[i] == 0;
    if (lead_zero) lens1[d - e[k - 1]] = d - e[k - 1];
  }
}

__global__ void k_tables(int k, int d, int side, const double* __restrict__ clo, const double* __restrict__ chi,
                         double* __restrict__ packed, int2* __restrict__ ttab, int32_t* __restrict__ lens2,
                         int32_t* __restrict__ lens1, int32_t* __restrict__ padlist) {
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  tables_entry(f, k, d, side, clo, chi, packed, ttab, lens2, lens1, padlist);
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

// ---------------------------------------------------------------------------
// Stage 1.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_uniform(double x) {
  const int64_t b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffff));
  const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
  return __longlong_as_double(((int64_t)hi << 32) | (uint32_t)lo);
}

// The packed rows are read from global memory (a generic pointer would make
// every load a flat load, which also counts against the scalar-load counter).
typedef double gvec2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) const gvec2 gdouble2;

// Row r of the packed table starts at C(r+m, m+1) and holds C(r+m, m)
// tuples; the walk uses additions only: c_j = C(r+j, j) obeys
// c_j(r+1) = c_j(r) + c_{j-1}(r+1) (Pascal), so no division runs per row.
// Four rows are in flight in four register buffers that rotate in place (no
// copies, so waiting for one row never waits for the others).  Lanes whose chain has
// not started (|t| > r), and rows past d, read the zero entry the table keeps
// after its last row, so every load is unconditional.
template <int R, int CLS>
__device__ __forceinline__ void stage1_steps(const double2 c, const double (&u)[R], const double (&v)[R],
                                             const CellOps (&ops)[R], double (&nl)[R], double (&hh)[R]) {
#pragma unroll
  for (int j = 0; j < R; j++) {
    if (CLS == CLS_POS) step_pos(nl[j], hh[j], u[j], v[j], c.x, c.y);
    else if (CLS == CLS_NEG) step_neg(nl[j], hh[j], u[j], v[j], c.x, c.y);
    else step_gen(nl[j], hh[j], ops[j], c.x, c.y);
  }
}

// Advance the row walk by one row: returns the index to read for row `rl`
// (the zero entry for lanes whose chain has not started, or past the table).
template <int M>
__device__ __forceinline__ int64_t stage1_next(int64_t& off, int64_t& c1, int64_t& c2, int64_t& c3, int& rl,
                                               int d, int gdeg, int64_t gidx, int64_t zidx) {
  const int64_t at = (rl <= d && gdeg <= rl) ? off + gidx : zidx;
  off += M == 1 ? c1 : (M == 2 ? c2 : c3);
  c1 += 1;
  c2 += c1;
  c3 += c2;
  rl++;
  return at;
}

constexpr int STAGE1_PF = 8;

template <int R, int CLS, int M>
__device__ __forceinline__ void stage1_chain_m(const double2* __restrict__ Pg, int d, int r0, int gdeg, int64_t gidx,
                                               const double (&u)[R], const double (&v)[R], const CellOps (&ops)[R],
                                               double (&nl)[R], double (&hh)[R]) {
  constexpr int m = M;
  const gdouble2* P = (const gdouble2*)Pg;
  const int64_t zidx = dbinom(d + 1 + m, m + 1);  // zero entry after the last row
  int64_t c1 = r0 + 1, c2 = dbinom(r0 + 2, 2), c3 = dbinom(r0 + 3, 3);
  int64_t off = dbinom(r0 + m, m + 1);  // start of the next row to load
  int rl = r0;                          // that row's index
  // STAGE1_PF rows in flight; rows past d read the zero entry and are never used
  constexpr int PF = STAGE1_PF;
  gvec2 q[PF];
#pragma unroll
  for (int i = 0; i < PF; i++) q[i] = P[stage1_next<M>(off, c1, c2, c3, rl, d, gdeg, gidx, zidx)];
  int r = r0;
  for (; r + PF - 1 <= d; r += PF) {
#pragma unroll
    for (int i = 0; i < PF; i++) {
      stage1_steps<R, CLS>(make_double2(q[i].x, q[i].y), u, v, ops, nl, hh);
      q[i] = P[stage1_next<M>(off, c1, c2, c3, rl, d, gdeg, gidx, zidx)];
    }
  }
#pragma unroll
  for (int i = 0; i < PF - 1; i++)
    if (r + i <= d) stage1_steps<R, CLS>(make_double2(q[i].x, q[i].y), u, v, ops, nl, hh);
}

template <int R, int CLS>
__device__ __forceinline__ void stage1_chain(const double2* __restrict__ Pg, int m, int d, int r0, int gdeg,
                                             int64_t gidx, const double (&u)[R], const double (&v)[R],
                                             const CellOps (&ops)[R], double (&nl)[R], double (&hh)[R]) {
  if (m == 1) stage1_chain_m<R, CLS, 1>(Pg, d, r0, gdeg, gidx, u, v, ops, nl, hh);
  else if (m == 2) stage1_chain_m<R, CLS, 2>(Pg, d, r0, gdeg, gidx, u, v, ops, nl, hh);
  else stage1_chain_m<R, CLS, 3>(Pg, d, r0, gdeg, gidx, u, v, ops, nl, hh);
}

// Per-polynomial tables and stage outputs, passed by value; blockIdx.z (or a
// loop in the leaf kernel) selects the polynomial.
constexpr int PMAX = 8;

struct PolyTab {
  const double2* packed;   // stage-1 coefficients (k >= 2) or the leaf row (k == 1)
  const int2* ttab;        // graded tuple -> (|t|, output position)
  const int32_t* lens2;    // O_2 chain lengths (k == 4)
  const int32_t* padlist;  // zero slots of the padded stage-1 rows (k == 3)
  int d;
  int nt;                  // trailing tuples of stage 1: C(d+k-1, k-1)
  int npad;
};

// Node q's entry j sits at rows + q * stride + j * estride (doubles).  Rows
// written by stage 1 are node-major (estride = entry width); the leaf input
// written by a middle stage is entry-major (stride = LEAF_W, estride = LEAF_W *
// nodes),
// so the 64 lanes of a middle-stage wave, which are 64 consecutive nodes,
// store each entry contiguously, and leaf lanes of neighbouring columns read
// neighbouring addresses.
struct RowSet {
  double* rows[PMAX];
  int64_t stride[PMAX];
  int64_t estride[PMAX];
};

struct PolySet {
  int np;
  PolyTab p[PMAX];
};

template <int R, int CLS>
__device__ __forceinline__ void stage1_body(const PolyTab& pt, int m, const int32_t* __restrict__ labels0, int begin,
                                            int cnt, const AxisGrid& g, int64_t gidx, bool active, int gdeg,
                                            int opos, int r0, double* __restrict__ base, int64_t stride,
                                            int out_width) {
  double u[R], v[R], nl[R], hh[R];
  CellOps ops[R];
#pragma unroll
  for (int j = 0; j < R; j++) {
    const int32_t lab = labels0[begin + (j < cnt ? j : 0)];
    double cnl, chi;
    cell(g, lab, cnl, chi);
    ops[j] = cell_ops(cnl, chi, CLS);
    ops[j].u = wave_uniform(ops[j].u);
    ops[j].v = wave_uniform(ops[j].v);
    if (CLS == CLS_STRADDLE) {
      ops[j].nu = wave_uniform(ops[j].nu);
      ops[j].nv = wave_uniform(ops[j].nv);
    }
    u[j] = ops[j].u;
    v[j] = ops[j].v;
    nl[j] = 0.0;
    hh[j] = 0.0;
  }
  stage1_chain<R, CLS>(pt.packed, m, pt.d, r0, gdeg, gidx, u, v, ops, nl, hh);
  if (!active) return;
#pragma unroll
  for (int j = 0; j < R; j++) {
    if (j < cnt) {
      // 16-byte aligned (rows, strides and entries are): one store
      double* o = base + (int64_t)(begin + j) * stride + (int64_t)opos * out_width;
      *reinterpret_cast<double2*>(o) = make_double2(nl[j], hh[j]);
    }
  }
}

// One workgroup per (polynomial z, segment x, tuple wave y) item, y fastest.
// Items are dealt to the XCDs in chunks of whole segments (all tuple waves of
// one (z, x)): every entry of a segment's output rows is then written from
// one XCD, whose L2 merges the scattered 16-byte stores of the tuple waves
// into whole lines before they leave it (dealing whole tuple waves instead,
// which keeps each XCD on its share of the coefficients, measured 12 %
// slower: 202 against 178 us at level 10 of the curve).
template <int R>
__global__ __launch_bounds__(64) void k_stage1(PolySet ps, int m, const int32_t* __restrict__ labels0,
                                               const int4* __restrict__ seg, const int64_t* __restrict__ nseg,
                                               AxisGrid g, RowSet out, int out_width, int64_t maxseg, int ny,
                                               int64_t chunk, int64_t items) {
  round_up_mode();
  const int64_t item = xcd_item(blockIdx.x % NXCD, blockIdx.x / NXCD, chunk);
  if (item >= items) return;
  const int wy = (int)(item % ny);
  const int64_t sx = (item / ny) % maxseg;
  const int pz = (int)(item / (maxseg * ny));
  if (sx >= *nseg) return;
  const PolyTab& pt = ps.p[pz];
  const int nt = pt.nt, d = pt.d;
  const int ntw = (nt + 63) / 64;
  if (wy > ntw) return;
  if (wy == ntw) {  // zero the padding slots of this segment's rows
    if (pt.npad == 0) return;
    const int4 sg = seg[sx];
    double* base = out.rows[pz];
    const int64_t stride = out.stride[pz];
    for (int j = 0; j < sg.z; j++)
      for (int i = threadIdx.x; i < pt.npad; i += 64) {
        double* o = base + (int64_t)(sg.y + j) * stride + (int64_t)pt.padlist[i] * out_width;
        o[0] = 0.0;
        o[1] = 0.0;
      }
    return;
  }
  const int4 sg = seg[sx];
  const int begin = sg.y, cnt = sg.z, cls = sg.w;
  const int lane = threadIdx.x;
  const int64_t gidx = (int64_t)wy * 64 + lane;
  const bool active = gidx < nt;
  int gdeg = d + 1, opos = 0;
  if (active) {
    const int2 tt = pt.ttab[gidx];
    gdeg = tt.x;
    opos = tt.y;
  }
  const int r0 = __builtin_amdgcn_readfirstlane(gdeg);  // lane 0 holds the wave's smallest |t|
  double* base = out.rows[pz];
  const int64_t stride = out.stride[pz];
  if (cls == CLS_POS)
    stage1_body<R, CLS_POS>(pt, m, labels0, begin, cnt, g, gidx, active, gdeg, opos, r0, base, stride, out_width);
  else if (cls == CLS_NEG)
    stage1_body<R, CLS_NEG>(pt, m, labels0, begin, cnt, g, gidx, active, gdeg, opos, r0, base, stride, out_width);
  else  // cells containing 0 in their interior: rare, one node at a time
    for (int j = 0; j < cnt; j++)
      stage1_body<1, CLS_STRADDLE>(pt, m, labels0, begin + j, 1, g, gidx, active, gdeg, opos, r0, base, stride,
                                   out_width);
}

// ---------------------------------------------------------------------------
// Narrow stage.
// ---------------------------------------------------------------------------
// The parent row is consumed chain by chain in groups of NARROW_GROUP
// entries read with scalar loads.  A chain of n entries takes ceil(n/G)
// groups; its first group starts G*ceil(n/G) - n entries early (inside the
// previous chain, or in the slack before the first row) and those leading
// entries are replaced by zeros in scalar registers.  Every chain starts from
// J = 0, so each entry is one uniform interval step (0*I + c = c exactly, up
// to the sign of a zero) and the only per-chain work is one store.  The next
// group's loads are issued after the current group has arrived (a data
// dependency through `after`), so they overlap the current group's steps;
// scalar loads complete out of order, and waiting for the current group must
// not also wait for the next one.
constexpr int NARROW_GROUP = 8;

constexpr int SPLIT_MAX = 16;

struct ChainSplit {
  int n;
  int j0[SPLIT_MAX + 1];      // first chain of group g (j0[n] = number of chains)
  int64_t p0[SPLIT_MAX + 1];  // first row entry of group g
};

// Zero that the compiler can only produce once `x` is available.
__device__ __forceinline__ int64_t after(double x) {
  int64_t z;
  asm volatile("s_mov_b64 %0, 0" : "=s"(z) : "s"(x));
  return z;
}

template <bool ORDER1>
__device__ __forceinline__ int chain_len(const int32_t* __restrict__ lens, int j) {
  return ORDER1 ? j : lens[j];
}

// Rows read by a narrow stage are never written during the launch; the
// constant address space lets the compiler fetch the wave-uniform stream with
// scalar loads.
typedef double dvec2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(4))) const dvec2 crow_t;

template <int CLS, bool ORDER1>
__device__ __forceinline__ void narrow_run(const crow_t* __restrict__ C, const int32_t* __restrict__ lens, int j,
                                           const int jend, int64_t cpos, const CellOps& o, bool valid,
                                           double* __restrict__ out, int64_t es, int out_width) {
  constexpr int G = NARROW_GROUP;
  if (j >= jend) return;
  int n = chain_len<ORDER1>(lens, j) + 1;  // entries of chain j
  int ng = (n + G - 1) / G;                // its groups
  int g = 0;                               // current group within the chain
  int64_t gpos = cpos - (G * ng - n);      // first entry of the current group
  dvec2 A[G];
#pragma unroll
  for (int e = 0; e < G; e++) A[e] = C[gpos + e];
  double nl = 0.0, hh = 0.0;
  while (true) {
    // next group coordinates
    int jn = j, gn = g + 1, nn = n, ngn = ng;
    int64_t cposn = cpos, gposn = gpos + G;
    if (gn == ng) {
      jn = j + 1;
      cposn = cpos + n;
      gn = 0;
      if (jn < jend) {
        nn = chain_len<ORDER1>(lens, jn) + 1;
        ngn = (nn + G - 1) / G;
        gposn = cposn - (G * ngn - nn);
      }
    }
    const bool more = jn < jend;
    const int64_t z = after(A[0].x);
    dvec2 B[G];
    if (more) {
#pragma unroll
      for (int e = 0; e < G; e++) B[e] = C[gposn + z + e];
    }
    if (g == 0) {
      const int pad = G * ng - n;
#pragma unroll
      for (int e = 0; e < G; e++)
        if (e < pad) A[e] = dvec2{0.0, 0.0};
    }
#pragma unroll
    for (int e = 0; e < G; e++) {
      if (CLS == CLS_POS) step_pos(nl, hh, o.u, o.v, A[e].x, A[e].y);
      else if (CLS == CLS_NEG) step_neg(nl, hh, o.u, o.v, A[e].x, A[e].y);
      else step_gen(nl, hh, o, A[e].x, A[e].y);
    }
    if (g == ng - 1) {
      if (valid) {
        // 16-byte aligned rows, strides and entries: one store
        *reinterpret_cast<double2*>(out + (int64_t)j * es) = make_double2(nl, hh);
      }
      nl = 0.0;
      hh = 0.0;
    }
    if (!more) break;
#pragma unroll
    for (int e = 0; e < G; e++) A[e] = B[e];
    j = jn; g = gn; n = nn; ng = ngn; cpos = cposn; gpos = gposn;
  }
}

// Middle stage on padded rows (k = 3): every group of 8 entries belongs to one
// chain, chains end on group boundaries, and the leading zeros replace the
// masking; two register buffers alternate so no copies are needed.
typedef __attribute__((address_space(1))) const dvec2 vrow_t;

// ROW = crow_t: the row is wave-uniform (scalar loads, the next group issued
// once the current one has arrived); ROW = vrow_t: every lane reads its own
// parent's row with vector loads.
//
// Scalar rows are also pulled into L2 ahead of the scalar loads: at every
// eighth group the wave loads the first dword of each 16-byte entry of the
// 64-entry block that starts 8 groups later straight into a scratch corner
// of LDS (global_load_lds: no register waits for it, nothing reads it), so
// that the scalar loads of those groups find the lines in L2 rather than
// waiting on HBM.  The wave waits for those loads before it leaves.
#ifndef VX_NARROW_PREFETCH
#define VX_NARROW_PREFETCH 1
#endif
template <int CLS, class ROW>
__device__ __forceinline__ void narrow_padded(ROW* __restrict__ C, int j, const int jend, const CellOps& o,
                                              bool valid, double* __restrict__ out, int64_t es, int out_width) {
  constexpr bool SCALAR = __is_same(ROW, crow_t);
  constexpr bool PREFETCH = SCALAR && VX_NARROW_PREFETCH;
  // vector rows move half groups (chains still end on whole PADG groups), so
  // that the two register buffers cost 32 VGPRs, not 64
  constexpr int G = SCALAR ? PADG : PADG / 2;
  constexpr int GM = PADG / G;
  if (j >= jend) return;
  // 32-bit group counters: the scalar unit compares 32-bit values only
  int g = (int)padded_groups(j) * GM;
  int gend = (int)padded_groups(j + 1) * GM;
  const int glast = (int)padded_groups(jend) * GM;
  dvec2 A[G], B[G];
#pragma unroll
  for (int e = 0; e < G; e++) A[e] = C[(int64_t)g * G + e];
  double nl = 0.0, hh = 0.0;
  auto steps = [&](const dvec2 (&X)[G]) {
#pragma unroll
    for (int e = 0; e < G; e++) {
      if (CLS == CLS_POS) step_pos(nl, hh, o.u, o.v, X[e].x, X[e].y);
      else if (CLS == CLS_NEG) step_neg(nl, hh, o.u, o.v, X[e].x, X[e].y);
      else step_gen(nl, hh, o, X[e].x, X[e].y);
    }
  };
  typedef __attribute__((address_space(1))) const double gdbl_t;
  typedef __attribute__((address_space(1))) const void gvoid_t;
  typedef __attribute__((address_space(3))) void lvoid_t;
  __shared__ int pf_lds[64];
  gdbl_t* V = reinterpret_cast<gdbl_t*>(reinterpret_cast<uintptr_t>(C));
  auto prefetch = [&]() {
    if (PREFETCH && (g & 7) == 0 && g + 16 <= glast)  // lane l: entry l of the block, every line of it
      __builtin_amdgcn_global_load_lds((gvoid_t*)(V + 2 * ((int64_t)(g + 8) * G + threadIdx.x)), (lvoid_t*)pf_lds,
                                       4, 0, 0);
  };
  auto finish = [&]() {
    g++;
    if (g == gend) {
      if (valid) {
        // 16-byte aligned rows, strides and entries: one store
        *reinterpret_cast<double2*>(out + (int64_t)j * es) = make_double2(nl, hh);
      }
      nl = 0.0;
      hh = 0.0;
      j++;
      gend = (int)padded_groups(j + 1) * GM;
    }
  };
  while (true) {
    {
      const int64_t z = SCALAR ? after(A[0].x) : 0;
      const bool more = g + 1 < glast;
      if (more) {
#pragma unroll
        for (int e = 0; e < G; e++) B[e] = C[(int64_t)(g + 1) * G + z + e];
      }
      prefetch();
      steps(A);
      finish();
      if (!more) break;
    }
    {
      const int64_t z = SCALAR ? after(B[0].x) : 0;
      const bool more = g + 1 < glast;
      if (more) {
#pragma unroll
        for (int e = 0; e < G; e++) A[e] = C[(int64_t)(g + 1) * G + z + e];
      }
      prefetch();
      steps(B);
      finish();
      if (!more) break;
    }
  }
  if (PREFETCH) __builtin_amdgcn_s_waitcnt(0x0f70);  // vmcnt(0): no LDS write in flight when the wave ends
}

// Padded rows (k = 3): split g of n splits the chains 0..d into runs of about
// equal group counts; its first chain is the first j with padded_groups(j) >=
// padded_groups(d + 1) * g / n (split n ends at d + 1).  Wave-uniform.
__device__ __forceinline__ int padded_split(int d, int g, int n) {
  if (g >= n) return d + 1;
  const int64_t target = (padded_groups(d + 1) * g + n - 1) / n;
  int lo = 0, hi = d + 1;  // padded_groups(hi) >= target
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (padded_groups(mid) >= target) hi = mid; else lo = mid + 1;
  }
  return __builtin_amdgcn_readfirstlane(lo);
}

// The chains of split gi of gdim on a wave-uniform padded row.
__device__ __forceinline__ void narrow_scalar_split(const crow_t* __restrict__ C, int d, int gi, int gdim, int cls,
                                                    const CellOps& o, bool valid, double* __restrict__ w, int64_t es,
                                                    int out_width) {
  const int j0 = padded_split(d, gi, gdim), j1 = padded_split(d, gi + 1, gdim);
  if (cls == CLS_POS) narrow_padded<CLS_POS, crow_t>(C, j0, j1, o, valid, w, es, out_width);
  else if (cls == CLS_NEG) narrow_padded<CLS_NEG, crow_t>(C, j0, j1, o, valid, w, es, out_width);
  else narrow_padded<CLS_STRADDLE, crow_t>(C, j0, j1, o, valid, w, es, out_width);
}

struct SplitSet {
  ChainSplit s[PMAX];
};

// One workgroup per (polynomial, segment, chain group) item, items ordered
// with the chain group fastest and dealt to the XCDs in chunks, so that the
// segments of one parent, which stream the same parent row, share an L2.
constexpr int NARROW_XCD_CHUNK = 64;

template <bool ORDER1, bool PADDED>
__global__ __launch_bounds__(64) void k_narrow(PolySet ps, RowSet in, SplitSet splits,
                                               const int32_t* __restrict__ labels, const int4* __restrict__ seg,
                                               const int64_t* __restrict__ nseg, AxisGrid g, RowSet out,
                                               int out_width, int64_t maxseg, int gdim, int64_t items) {
  round_up_mode();
  const int64_t item = xcd_item(blockIdx.x % NXCD, blockIdx.x / NXCD, NARROW_XCD_CHUNK);
  if (item >= items) return;
  const int gi = (int)(item % gdim);
  const int64_t sidx = (item / gdim) % maxseg;
  const int pz = (int)(item / ((int64_t)gdim * maxseg));
  if (sidx >= *nseg) return;
  const ChainSplit& split = splits.s[pz];
  if (!PADDED && gi >= split.n) return;
  const int4 sg = seg[sidx];
  const int parent = sg.x, begin = sg.y, cnt = sg.z, cls = sg.w;
  const int lane = threadIdx.x;
  const bool valid = lane < cnt;
  const int64_t node = begin + (valid ? lane : 0);
  double cnl, chi;
  cell(g, labels[node], cnl, chi);
  const CellOps o = cell_ops(cnl, chi, cls);
  const crow_t* C = (const crow_t*)(in.rows[pz] + (int64_t)parent * in.stride[pz]);
  double* w = out.rows[pz] + node * out.stride[pz];
  const int64_t es = out.estride[pz];
  const int32_t* lens = ps.p[pz].lens2;
  if (PADDED) {
    narrow_scalar_split(C, ps.p[pz].d, gi, gdim, cls, o, valid, w, es, out_width);
    return;
  }
  const int j0 = __builtin_amdgcn_readfirstlane(split.j0[gi]);
  const int j1 = __builtin_amdgcn_readfirstlane(split.j0[gi + 1]);
  const int64_t p0 = split.p0[gi];
  if (cls == CLS_POS) narrow_run<CLS_POS, ORDER1>(C, lens, j0, j1, p0, o, valid, w, es, out_width);
  else if (cls == CLS_NEG) narrow_run<CLS_NEG, ORDER1>(C, lens, j0, j1, p0, o, valid, w, es, out_width);
  else narrow_run<CLS_STRADDLE, ORDER1>(C, lens, j0, j1, p0, o, valid, w, es, out_width);
}

// Packed middle-stage waves (k = 3): the 64 lanes take consecutive entries of
// one sign class's tail list, so a wave holds nodes of several parents and
// every lane streams its own parent's row with vector loads (the rows of
// consecutive tails are neighbours, so a load instruction touches a few
// cache lines).
struct TailLists {
  const int32_t* node[2];  // NEG, POS
  const int32_t* par[2];
};

// Packed waves with at most PK_SLOTS distinct parents (the usual case) stage
// every group of 8 entries of those parents' rows in LDS: lanes 0 .. 8P-1
// load one entry each (issued a group ahead, written to LDS after the
// current group's steps), and every lane reads its parent's entries from
// LDS.  One wave per workgroup, so the in-order LDS queue of the wave orders
// the writes before the next group's reads.
constexpr int PK_SLOTS = 8;

template <int CLS>
__device__ __forceinline__ void narrow_packed_lds(const double* __restrict__ rows, int64_t stride, int slot, int nslot,
                                                  const int32_t* __restrict__ spar, int j, const int jend,
                                                  const CellOps& o, bool valid, double* __restrict__ out, int64_t es,
                                                  int out_width) {
  constexpr int G = PADG;
  __shared__ dvec2 buf[2][PK_SLOTS][G];
  if (j >= jend) return;
  const int lane = threadIdx.x;
  const bool loader = lane < G * nslot;
  const int ls = loader ? lane / G : 0, le = lane % G;
  const vrow_t* src = (const vrow_t*)(rows + (int64_t)spar[ls] * stride) + le;
  int g = (int)padded_groups(j);
  int gend = (int)padded_groups(j + 1);
  const int glast = (int)padded_groups(jend);
  if (loader) buf[0][ls][le] = src[(int64_t)g * G];
  int b = 0;
  double nl = 0.0, hh = 0.0;
  while (true) {
    const bool more = g + 1 < glast;
    dvec2 nxt = dvec2{0.0, 0.0};
    if (more && loader) nxt = src[(int64_t)(g + 1) * G];
#pragma unroll
    for (int e = 0; e < G; e++) {
      const dvec2 x = buf[b][slot][e];
      if (CLS == CLS_POS) step_pos(nl, hh, o.u, o.v, x.x, x.y);
      else step_neg(nl, hh, o.u, o.v, x.x, x.y);
    }
    g++;
    if (g == gend) {
      if (valid) {
        // 16-byte aligned rows, strides and entries: one store
        *reinterpret_cast<double2*>(out + (int64_t)j * es) = make_double2(nl, hh);
      }
      nl = 0.0;
      hh = 0.0;
      j++;
      gend = (int)padded_groups(j + 1);
    }
    if (!more) break;
    b ^= 1;
    if (loader) buf[b][ls][le] = nxt;
  }
}

__device__ __forceinline__ void narrow_packed_item(const PolySet& ps, const RowSet& in, const int32_t* labels,
                                                   const int4& sg, const TailLists& tl, const AxisGrid& g,
                                                   const RowSet& out, int out_width, int pz, int gi, int gdim) {
  const int cnt = sg.z, cls = sg.w;
  const int lane = threadIdx.x;
  const bool valid = lane < cnt;
  const int64_t ti = sg.x + (valid ? lane : 0);
  const int c = cls == CLS_NEG ? 0 : 1;
  const int64_t node = tl.node[c][ti], parent = tl.par[c][ti];
  double cnl, chi;
  cell(g, labels[node], cnl, chi);
  const CellOps o = cell_ops(cnl, chi, cls);
  double* w = out.rows[pz] + node * out.stride[pz];
  const int64_t es = out.estride[pz];
  const int d = ps.p[pz].d;
  const int j0 = padded_split(d, gi, gdim), j1 = padded_split(d, gi + 1, gdim);
  // parent slots: the parents of a packed segment ascend with the lane
  const int64_t prev = __shfl_up(parent, 1);
  const bool first = lane == 0 || parent != prev;
  const uint64_t fm = __ballot(first);
  const int nslot = __popcll(fm);
  if (nslot <= PK_SLOTS) {
    __shared__ int32_t spar[PK_SLOTS];
    const int slot = __popcll(fm & ((2ull << lane) - 1)) - 1;
    if (first) spar[slot] = (int32_t)parent;
    if (cls == CLS_NEG)
      narrow_packed_lds<CLS_NEG>(in.rows[pz], in.stride[pz], slot, nslot, spar, j0, j1, o, valid, w, es, out_width);
    else
      narrow_packed_lds<CLS_POS>(in.rows[pz], in.stride[pz], slot, nslot, spar, j0, j1, o, valid, w, es, out_width);
    return;
  }
  vrow_t* C = (vrow_t*)(in.rows[pz] + parent * in.stride[pz]);
  if (cls == CLS_NEG) narrow_padded<CLS_NEG, vrow_t>(C, j0, j1, o, valid, w, es, out_width);
  else narrow_padded<CLS_POS, vrow_t>(C, j0, j1, o, valid, w, es, out_width);
}

// k = 3 with packed tails: one launch over the parent-uniform segments and
// the packed ones (flagged), so that vector-load waves share the CUs with
// scalar-load waves and run next to the segments that read the same rows.
__global__ __launch_bounds__(64) void k_narrow_mixed(PolySet ps, RowSet in, const int32_t* __restrict__ labels,
                                                     const int4* __restrict__ seg, const int64_t* __restrict__ nfull,
                                                     const int64_t* __restrict__ nseg, TailLists tl, AxisGrid g,
                                                     RowSet out, int out_width, int64_t maxseg, int gdim,
                                                     int64_t items) {
  round_up_mode();
  const int64_t item = xcd_item(blockIdx.x % NXCD, blockIdx.x / NXCD, NARROW_XCD_CHUNK);
  if (item >= items) return;
  const int gi = (int)(item % gdim);
  const int64_t t = (item / gdim) % maxseg;
  const int pz = (int)(item / ((int64_t)gdim * maxseg));
  (void)nfull;
  if (t >= *nseg) return;
  const int4 sg = seg[t];
  if (sg.w & SEG_PACKED) {
    narrow_packed_item(ps, in, labels, make_int4(sg.x, sg.y, sg.z, sg.w & ~SEG_PACKED), tl, g, out, out_width, pz,
                       gi, gdim);
    return;
  }
  const int parent = sg.x, begin = sg.y, cnt = sg.z, cls = sg.w;
  const int lane = threadIdx.x;
  const bool valid = lane < cnt;
  const int64_t node = begin + (valid ? lane : 0);
  double cnl, chi;
  cell(g, labels[node], cnl, chi);
  const CellOps o = cell_ops(cnl, chi, cls);
  const crow_t* C = (const crow_t*)(in.rows[pz] + (int64_t)parent * in.stride[pz]);
  double* w = out.rows[pz] + node * out.stride[pz];
  const int64_t es = out.estride[pz];
  narrow_scalar_split(C, ps.p[pz].d, gi, gdim, cls, o, valid, w, es, out_width);
}

// ---------------------------------------------------------------------------
// Leaf stage and exclusion test.
//
// A lane whose cell is NEG evaluates the mirrored polynomial
// Ft(y) = F(-y) = sum (-1)^e c_e y^e on the nonnegative cell -I with the POS
// formula.  Negation is exact and commutes with outward rounding, so every
// intermediate value is (-1)^e times the direct one and the final value (e=0)
// is identical.  (-1)^e c_e for odd e is the pair (nlo, hi) read swapped,
// (hi, nlo).
// ---------------------------------------------------------------------------
typedef double dpair_a8 __attribute__((ext_vector_type(2), aligned(8)));

// General (straddling) leaf chain for one box; entry j at R + es * j.
__device__ __forceinline__ void leaf_chain_gen(const double* __restrict__ R, int64_t es, int d, double cnl,
                                               double chi, double& nl, double& hh) {
  const CellOps o = cell_ops(cnl, chi, CLS_STRADDLE);
  nl = R[0];
  hh = R[1];
  for (int j = 1; j <= d; j++) step_gen(nl, hh, o, R[es * j], R[es * j + 1]);
}

// Up to LR boxes of one column and one sign class (POS or NEG) share every
// coefficient load.  Entry j (exponent d - j) is the pair (nlo, hi) at
// R + es * j; mirrored (NEG) boxes take it swapped, (hi, nlo), when d - j is
// odd (a per-lane select after the load, once per entry for all LR boxes).
// PF entries are in flight, so entries up to max(PF, d + PF) are read (the
// buffers are sized for LEAF_PF_MAX); those past d are never used.
constexpr int LEAF_PF_MAX = 8;

// DODD = d is odd (then the even entries are the odd exponents).
template <int LR, int PF, bool DODD>
__device__ __forceinline__ void leaf_chains_p(const double* __restrict__ R, int64_t es, int d, bool sh,
                                              const double (&u)[LR], const double (&v)[LR], double (&nl)[LR],
                                              double (&hh)[LR]) {
  static_assert(PF % 2 == 0 && PF <= LEAF_PF_MAX, "even prefetch depth within the row slack");
  // swap of even entries (d - j odd iff d odd) and of odd entries (iff d even)
  const bool swe = DODD && sh, swo = !DODD && sh;
  auto at = [&](int j) -> dpair_a8 { return *reinterpret_cast<const dpair_a8*>(R + es * j); };
  auto fix = [](const dpair_a8& x, bool sw) -> dpair_a8 { return sw ? dpair_a8{x.y, x.x} : x; };
  const dpair_a8 c = fix(at(0), swe);
#pragma unroll
  for (int i = 0; i < LR; i++) {
    nl[i] = c.x;
    hh[i] = c.y;
  }
  dpair_a8 q[PF];
#pragma unroll
  for (int i = 0; i < PF; i++) q[i] = at(1 + i);
  auto steps = [&](const dpair_a8& x) {
#pragma unroll
    for (int i = 0; i < LR; i++) step_pos(nl[i], hh[i], u[i], v[i], x.x, x.y);
  };
  // every call site has j = 1 + (even) + i with i known, so the parity is static
  int j = 1;
  for (; j + PF - 1 <= d; j += PF) {
#pragma unroll
    for (int i = 0; i < PF; i++) {
      steps(fix(q[i], (i & 1) ? swe : swo));
      q[i] = at(j + PF + i);
    }
  }
#pragma unroll
  for (int i = 0; i < PF - 1; i++)
    if (j + i <= d) steps(fix(q[i], (i & 1) ? swe : swo));
}

template <int LR, int PF>
__device__ __forceinline__ void leaf_chains(const double* __restrict__ R, int64_t es, int d, int sh,
                                            const double (&u)[LR], const double (&v)[LR], double (&nl)[LR],
                                            double (&hh)[LR]) {
  if (d & 1) leaf_chains_p<LR, PF, true>(R, es, d, sh != 0, u, v, nl, hh);
  else leaf_chains_p<LR, PF, false>(R, es, d, sh != 0, u, v, nl, hh);
}

// One lane per leaf segment (<= LR boxes of one parent and one class; LR =
// LEAF_R, or 1 on the smallest levels, where the lanes are plentiful and
// each lane's serial chain is the latency).
// SPLITP: the polynomials of a segment run on P2 adjacent lanes (P2 = the
// power of two >= np), one each, and the lanes OR their exclusion flags with
// cross-lane shuffles; small levels use it to halve (or better) the serial
// chain of each lane.
constexpr int LEAF_R = 4;

// The large-level form (PF = 4) is held to 80 VGPRs (6 waves per SIMD
// instead of 4; it fits without spilling); the others keep their registers.
// alive (may be null; the last launch over the polynomials only): set to 1
// for the parent of every box that keeps keep != 0 (cleared beforehand by the
// segment kernels); lanes of one parent may store concurrently, all the value 1.
template <bool SPLITP, int PF, int LR>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(PF == 4 ? 6 : 1, 8))) void k_leaf(PolySet ps, RowSet rows, const int4* __restrict__ seg,
                                              const int64_t* __restrict__ nseg, const int32_t* __restrict__ labels,
                                              int64_t nleaf, AxisGrid g, double* __restrict__ lo_out,
                                              double* __restrict__ hi_out, uint8_t* __restrict__ keep, int first,
                                              int p2, uint8_t* __restrict__ alive) {
  round_up_mode();
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t sid = SPLITP ? q / p2 : q;
  const int pl = SPLITP ? (int)(q % p2) : 0;
  if (sid >= *nseg) return;  // all p2 lanes of a segment leave together
  const int4 sg = seg[sid];
  const int64_t par = sg.x, begin = sg.y;
  const int cnt = sg.z, cls = sg.w;
  double u[LR], v[LR];
#pragma unroll
  for (int i = 0; i < LR; i++) {
    double cnl, chi;
    cell(g, labels[begin + (i < cnt ? i : 0)], cnl, chi);
    const CellOps o = cell_ops(cnl, chi, cls == CLS_STRADDLE ? CLS_POS : cls);
    u[i] = o.u;
    v[i] = o.v;
  }
  int excl = 0;  // bit i: box i excluded by some polynomial
  const int pbeg = SPLITP ? pl : 0, pend = SPLITP ? (pl < ps.np ? pl + 1 : pl) : ps.np;
  for (int p = pbeg; p < pend; p++) {
    const double* R = rows.rows[p] + par * rows.stride[p];
    const int64_t es = rows.estride[p];
    const int d = ps.p[p].d;
    double nl[LR], hh[LR];
    if (cls == CLS_STRADDLE) {
#pragma unroll
      for (int i = 0; i < LR; i++) {
        nl[i] = 0.0;
        hh[i] = 0.0;
        if (i < cnt) {
          double cnl, chi;
          cell(g, labels[begin + i], cnl, chi);
          leaf_chain_gen(R, es, d, cnl, chi, nl[i], hh[i]);
        }
      }
    } else {
      leaf_chains<LR, PF>(R, es, d, cls == CLS_NEG ? 1 : 0, u, v, nl, hh);
    }
#pragma unroll
    for (int i = 0; i < LR; i++) {
      if (i < cnt) {
        const double lo = -opaque(nl[i]);
        lo_out[p * nleaf + begin + i] = lo;
        hi_out[p * nleaf + begin + i] = hh[i];
        if ((lo > 0.0) || (hh[i] < 0.0)) excl |= 1 << i;
      }
    }
  }
  if (SPLITP) {
    for (int off = 1; off < p2; off <<= 1) excl |= __shfl_xor(excl, off);
    if (pl != 0) return;
  }
  if (keep) {
    bool any = false;
#pragma unroll
    for (int i = 0; i < LR; i++) {
      const bool ex = (excl >> i) & 1;
      if (i < cnt) {
        const uint8_t kv = first ? (ex ? 0 : 1) : (ex ? 0 : keep[begin + i]);
        keep[begin + i] = kv;
        any = any || kv != 0;
      }
    }
    if (alive && any) alive[par] = 1;
  }
}

// Largest leaf count for the one-polynomial-per-lane leaf launch, and for
// one box per lane.
#ifndef VX_LEAF_SPLIT_NODES
#define VX_LEAF_SPLIT_NODES (1536 * 1024)
#endif
constexpr int64_t LEAF_SPLIT_NODES = VX_LEAF_SPLIT_NODES;
constexpr int64_t LEAF_ONE_NODES = 16384;

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------
static AxisGrid make_grid(const double* dom, int axis, int level, int centre = 0) {
  AxisGrid g;
  g.dlo = dom[2 * axis];
  g.dhi = dom[2 * axis + 1];
  g.ndlo = -g.dlo;
  g.ndhi = -g.dhi;
  g.level = level;
  g.centre = centre;
  return g;
}

constexpr int64_t ROW_PAD = 16;  // entries of slack before and after every rows buffer

// Segments of one depth: runs of at most Z children of one parent and one
// sign class.  With `pack` (the middle stage of k = 3 on large levels), a
// class run of c children gives floor(c / Z) full segments and its c mod Z
// tail children go to a per-class tail list; the tails of all parents are
// then cut into "packed" segments of Z children of several parents each
// (class | SEG_PACKED), stored in parent order among the nfull
// parent-uniform ones.
struct SegPlan {
  int4* seg = nullptr;
  int64_t* nseg = nullptr;
  int64_t* cnt = nullptr;
  int64_t* off = nullptr;
  int64_t* bounds = nullptr;
  int64_t* tiles = nullptr;
  int64_t nparent = 0, nchild = 0, maxseg = 0;
  int Z = 64;
  int pack = 0;
  int64_t* nfull = nullptr;                    // parent-uniform segments (pack)
  int64_t* tcnt[2] = {};                       // tail children per parent, NEG / POS
  int64_t* toff[2] = {};                       // their exclusive scans
  int64_t* ttot[2] = {};                       // tail list lengths
  int64_t* ttiles[2] = {};
  int32_t* tnode[2] = {};                      // tail lists: node, parent
  int32_t* tpar[2] = {};
  int64_t maxpacked = 0;
};

static void plan_segments(Arena& A, SegPlan& sp, int64_t nparent, int64_t nchild, int Z, int pack = 0) {
  sp.nparent = nparent;
  sp.nchild = nchild;
  sp.Z = Z;
  sp.pack = pack;
  sp.maxseg = (nchild + Z - 1) / Z + 3 * nparent + 2;
  sp.seg = A.take<int4>(sp.maxseg > 0 ? sp.maxseg : 1);
  sp.nseg = A.take<int64_t>(1);
  sp.cnt = A.take<int64_t>(nparent + 1);
  sp.off = A.take<int64_t>(nparent + 1);
  sp.bounds = A.take<int64_t>(2 * nparent + 2);
  sp.tiles = A.take<int64_t>(scan_tiles(nparent));
  if (pack) {
    sp.nfull = A.take<int64_t>(1);
    sp.maxpacked = (nchild + Z - 1) / Z + 2;
    for (int c = 0; c < 2; c++) {
      sp.tcnt[c] = A.take<int64_t>(nparent + 1);
      sp.toff[c] = A.take<int64_t>(nparent + 1);
      sp.ttot[c] = A.take<int64_t>(1);
      sp.ttiles[c] = A.take<int64_t>(scan_tiles(nparent));
      sp.tnode[c] = A.take<int32_t>(nchild > 0 ? nchild : 1);
      sp.tpar[c] = A.take<int32_t>(nchild > 0 ? nchild : 1);
    }
  }
}

// Small levels: one workgroup builds the segments of every depth in a single
// launch (count, scan, write per depth); the larger levels use the 1-D grid
// kernels below.  Both write the same segments.
constexpr int64_t SMALL_LEVEL_NODES = 32768;  // largest depth count for the one-workgroup paths

struct SegJob {
  const int32_t* ptr[VX_KMAX];
  const int32_t* labels[VX_KMAX];
  AxisGrid g[VX_KMAX];
  int Z[VX_KMAX];
  int64_t nparent[VX_KMAX], nchild[VX_KMAX];
  int64_t* cnt[VX_KMAX];
  int64_t* bounds[VX_KMAX];
  int64_t* off[VX_KMAX];
  int4* seg[VX_KMAX];
  int64_t* nseg[VX_KMAX];
  int pl;  // the packed depth, -1 for none (large-level path only)
  int64_t* nfull;
  int64_t* tcnt[2];
  int64_t* toff[2];
  int64_t* ttot[2];
  int32_t* tnode[2];
  int32_t* tpar[2];
  uint8_t* alive;  // cleared per parent of the leaf depth (may be null)
};

constexpr int SMALL_THREADS = 1024;

// Item i of the (depth, parent) items of every depth, depth-major.
__device__ __forceinline__ int seg_item(const SegJob& J, int k, int64_t i, int64_t& p) {
  int l = 0;
  while (l + 1 < k && i >= J.nparent[l]) i -= J.nparent[l++];
  p = i;
  return l;
}

// Three phases over all depths at once: class bounds and segment counts of
// every (depth, parent) item, the per-depth scans, the segment records.
__global__ __launch_bounds__(SMALL_THREADS) void k_segments_small(int k, SegJob J) {
  round_up_mode();
  int64_t items = 0;
  for (int l = 0; l < k; l++) items += J.nparent[l];
  for (int64_t i = threadIdx.x; i < items; i += SMALL_THREADS) {
    int64_t p;
    const int l = seg_item(J, k, i, p);
    const int32_t* ptr = J.ptr[l];
    const int Z = J.Z[l];
    const int64_t b = ptr ? ptr[p] : 0, e = ptr ? ptr[p + 1] : J.nchild[l];
    int64_t ne, pb;
    class_bounds(J.labels[l], b, e, J.g[l], ne, pb);
    J.bounds[l][2 * p] = ne;
    J.bounds[l][2 * p + 1] = pb;
    J.cnt[l][p] = cdiv(ne - b, Z) + cdiv(pb - ne, Z) + cdiv(e - pb, Z);
    if (J.alive && l == k - 1) J.alive[p] = 0;
  }
  __syncthreads();
  constexpr int64_t TILE = (int64_t)SMALL_THREADS * SCAN_ITEMS;
  for (int l = 0; l < k; l++) {
    const int64_t np = J.nparent[l];
    int64_t carry = 0;
    for (int64_t base = 0; base < np; base += TILE) {
      const int64_t i0 = base + (int64_t)threadIdx.x * SCAN_ITEMS;
      int64_t v[SCAN_ITEMS];
      int64_t sum = 0;
#pragma unroll
      for (int j = 0; j < SCAN_ITEMS; j++) {
        v[j] = i0 + j < np ? J.cnt[l][i0 + j] : 0;
        sum += v[j];
      }
      int64_t tot;
      int64_t run = carry + block_exclusive_scan<SMALL_THREADS>(sum, tot);
#pragma unroll
      for (int j = 0; j < SCAN_ITEMS; j++) {
        if (i0 + j < np) J.off[l][i0 + j] = run;
        run += v[j];
      }
      carry += tot;
    }
    if (threadIdx.x == 0) *J.nseg[l] = carry;
  }
  __syncthreads();
  const int cls[3] = {CLS_NEG, CLS_STRADDLE, CLS_POS};
  for (int64_t i = threadIdx.x; i < items; i += SMALL_THREADS) {
    int64_t p;
    const int l = seg_item(J, k, i, p);
    const int32_t* ptr = J.ptr[l];
    const int Z = J.Z[l];
    const int64_t b = ptr ? ptr[p] : 0, e = ptr ? ptr[p + 1] : J.nchild[l];
    const int64_t cuts[4] = {b, J.bounds[l][2 * p], J.bounds[l][2 * p + 1], e};
    int64_t o = J.off[l][p];
    for (int c = 0; c < 3; c++)
      for (int64_t q = cuts[c]; q < cuts[c + 1]; q += Z) {
        const int64_t cnt = cuts[c + 1] - q < Z ? cuts[c + 1] - q : Z;
        J.seg[l][o++] = make_int4((int)p, (int)q, (int)cnt, cls[c]);
      }
  }
}

// Large levels: the segments of every depth in five launches in total (count,
// three scan passes, write), the depths sharing one 1-D grid; they are
// independent, so their work overlaps.
__global__ void k_seg_count_all(DepthBlocks D, SegJob J) {
  round_up_mode();
  int64_t t;
  const int l = D.find(blockIdx.x, t);
  const int64_t p = t * blockDim.x + threadIdx.x;
  if (p >= J.nparent[l]) return;
  const int32_t* ptr = J.ptr[l];
  const int Z = J.Z[l];
  const int64_t b = ptr ? ptr[p] : 0, e = ptr ? ptr[p + 1] : J.nchild[l];
  int64_t ne, pb;
  class_bounds(J.labels[l], b, e, J.g[l], ne, pb);
  J.bounds[l][2 * p] = ne;
  J.bounds[l][2 * p + 1] = pb;
  if (J.alive && l == D.count - 1) J.alive[p] = 0;
  if (l == J.pl) {
    J.cnt[l][p] = (ne - b) / Z + cdiv(pb - ne, Z) + (e - pb) / Z;
    J.tcnt[0][p] = (ne - b) % Z;
    J.tcnt[1][p] = (e - pb) % Z;
  } else {
    J.cnt[l][p] = cdiv(ne - b, Z) + cdiv(pb - ne, Z) + cdiv(e - pb, Z);
  }
}

__global__ void k_seg_write_all(DepthBlocks D, SegJob J) {
  int64_t t;
  const int l = D.find(blockIdx.x, t);
  const int64_t p = t * blockDim.x + threadIdx.x;
  if (p >= J.nparent[l]) return;
  const int32_t* ptr = J.ptr[l];
  const int Z = J.Z[l];
  const int64_t b = ptr ? ptr[p] : 0, e = ptr ? ptr[p + 1] : J.nchild[l];
  const int64_t cuts[4] = {b, J.bounds[l][2 * p], J.bounds[l][2 * p + 1], e};
  const int cls[3] = {CLS_NEG, CLS_STRADDLE, CLS_POS};
  int64_t o = J.off[l][p];
  if (l != J.pl) {
    for (int c = 0; c < 3; c++)
      for (int64_t q = cuts[c]; q < cuts[c + 1]; q += Z) {
        const int64_t cnt = cuts[c + 1] - q < Z ? cuts[c + 1] - q : Z;
        J.seg[l][o++] = make_int4((int)p, (int)q, (int)cnt, cls[c]);
      }
    return;
  }
  // Packed depth, in parent order: this parent's full runs of Z, then the
  // packed segments whose first tail child is one of this parent's (so a
  // packed wave runs next to the full segments that read the same rows).  A
  // class's packed segment w starts at tail-list offset Z w; the packed
  // segments starting before this parent's tails number ceil(toff / Z).
  const int64_t cN = cdiv(J.toff[0][p], Z), cP = cdiv(J.toff[1][p], Z);
  const int64_t cN1 = cdiv(J.toff[0][p + 1], Z), cP1 = cdiv(J.toff[1][p + 1], Z);
  o += cN + cP;
  for (int c = 0; c < 3; c++) {
    const int64_t full_end = c == 1 ? cuts[2] : cuts[c] + (cuts[c + 1] - cuts[c]) / Z * Z;
    for (int64_t q = cuts[c]; q < full_end; q += Z) {
      const int64_t cnt = full_end - q < Z ? full_end - q : Z;
      J.seg[l][o++] = make_int4((int)p, (int)q, (int)cnt, cls[c]);
    }
    if (c != 1) {
      const int tl = c == 0 ? 0 : 1;
      int64_t w = J.toff[tl][p];
      for (int64_t q = full_end; q < cuts[c + 1]; q++, w++) {
        J.tnode[tl][w] = (int32_t)q;
        J.tpar[tl][w] = (int32_t)p;
      }
    }
  }
  // packed records (x = offset in the class's tail list)
  const int64_t tn = *J.ttot[0], tp = *J.ttot[1];
  for (int64_t w = cN; w < cN1; w++)
    J.seg[l][o++] = make_int4((int)(w * Z), 0, (int)(tn - w * Z < Z ? tn - w * Z : Z), CLS_NEG | SEG_PACKED);
  for (int64_t w = cP; w < cP1; w++)
    J.seg[l][o++] = make_int4((int)(w * Z), 0, (int)(tp - w * Z < Z ? tp - w * Z : Z), CLS_POS | SEG_PACKED);
  if (p == 0) *J.nseg[l] = *J.nfull + cdiv(tn, Z) + cdiv(tp, Z);
}

#ifndef VX_NARROW_TARGET_WAVES
#define VX_NARROW_TARGET_WAVES 16384
#endif
constexpr int64_t NARROW_TARGET_WAVES = VX_NARROW_TARGET_WAVES;

// Chain lengths of O_m (m = 1 or 2) in order, host side.
static std::vector<int> o_lengths(int m, int d) {
  std::vector<int> L;
  if (m == 1) {
    for (int j = 0; j <= d; j++) L.push_back(j);
  } else {
    // O_2 = for e_k = d..0: for e = d - e_k .. 0: (e, e_k); length d - e - e_k
    for (int ek = d; ek >= 0; ek--)
      for (int e = d - ek; e >= 0; e--) L.push_back(d - e - ek);
  }
  return L;
}

// Split the chains of O_m into at most `groups` contiguous runs of about
// equal row entries (entries of chain j = length + 1).
static ChainSplit chain_split(int m, int d, int groups) {
  const std::vector<int> L = o_lengths(m, d);
  int64_t total = 0;
  for (int v : L) total += v + 1;
  ChainSplit cs;
  memset(&cs, 0, sizeof cs);
  int64_t acc = 0;
  int g = 1;
  for (size_t j = 0; j < L.size() && g < groups; j++) {
    acc += L[j] + 1;
    if (acc * groups >= total * g && j + 1 < L.size()) {
      cs.j0[g] = (int)j + 1;
      cs.p0[g] = acc;
      g++;
    }
  }
  cs.n = g;
  cs.j0[g] = (int)L.size();
  cs.p0[g] = total;
  return cs;
}

static void plan_prepared(Arena& A, Prepared& Q, const vx_poly* P, int np) {
  const int k = P[0].k;
  Q.k = k;
  Q.np = np;
  for (int p = 0; p < np; p++) {
    const int d = P[p].degree;
    Q.d[p] = d;
    Q.dmax = d > Q.dmax ? d : Q.dmax;
    Q.packed[p] = A.take<double>((k == 1 ? LEAF_W * (int64_t)(d + 1) : 2 * ntup(k, d)) + 2 * ROW_PAD * 3);
    Q.ttab[p] = A.take<int2>(k >= 2 ? ntup(k - 1, d) : 1);
    Q.lens2[p] = A.take<int32_t>(k == 4 ? ntup(2, d) : 1);
    Q.lens1[p] = A.take<int32_t>(d + 1);
    Q.padlist[p] = A.take<int32_t>(k == 3 ? padded_npad(d) + 1 : 1);
  }
}

size_t prepared_bytes(const vx_poly* P, int np) {
  Arena A;
  Prepared Q;
  plan_prepared(A, Q, P, np);
  return A.off + 256;
}

int prepare_polys(const vx_poly* P, int np, void* ws, size_t ws_bytes, Prepared* out, hipStream_t st) {
  Arena A;
  A.base = reinterpret_cast<char*>(ws);
  A.size = ws_bytes;
  plan_prepared(A, *out, P, np);
  if (A.overflow) VX_FAIL(VX_ECAPACITY, "workspace too small for the coefficient tables");
  const int k = P[0].k;
  for (int p = 0; p < np; p++) {
    int64_t cube = 1;
    for (int i = 0; i < k; i++) cube *= P[p].side;
    hipLaunchKernelGGL(k_tables, dim3((unsigned)((cube + 255) / 256)), dim3(256), 0, st, k, P[p].degree, P[p].side,
                       P[p].c_lo, P[p].c_hi, out->packed[p], out->ttab[p], out->lens2[p], out->lens1[p],
                       out->padlist[p]);
    VX_CHECK_LAUNCH("k_tables");
  }
  return VX_OK;
}

Prepared prepared_subset(const Prepared& Q, const int* idx, int n) {
  Prepared R;
  R.k = Q.k;
  R.np = n;
  for (int i = 0; i < n; i++) {
    const int p = idx[i];
    R.packed[i] = Q.packed[p];
    R.ttab[i] = Q.ttab[p];
    R.lens2[i] = Q.lens2[p];
    R.lens1[i] = Q.lens1[p];
    R.padlist[i] = Q.padlist[p];
    R.d[i] = Q.d[p];
    R.dmax = R.d[i] > R.dmax ? R.d[i] : R.dmax;
  }
  return R;
}

// Middle-stage node count from which tails are packed into full waves.
constexpr int64_t PACK_MIN_NODES = 8192;

struct EvalPlan {
  int k = 0;
  double* rows[VX_KMAX][VX_MAXPOLY] = {};  // output rows of stage l for polynomial p
  SegPlan seg[VX_KMAX];
  int R = 8;
  int mode[VX_KMAX] = {};  // per axis: 0 cells, 1 cell centres, 2 grid vertices (AxisGrid::centre)
};

#ifndef VX_STAGE1_RMAX
#define VX_STAGE1_RMAX 8
#endif
static int stage1_blocking(int64_t n0) {
  const int r = n0 <= 4 ? 1 : n0 <= 16 ? 2 : n0 <= 64 ? 4 : 8;
  return r < VX_STAGE1_RMAX ? r : VX_STAGE1_RMAX;
}

// Level workspace (measure with A.base == nullptr).  With `bound` the plan
// takes the largest choices at every depth (one node per segment, tail lists
// planned): its size is then monotone in the node counts, so a plan for upper
// bounds of the counts covers every smaller level.
static void plan_eval(Arena& A, EvalPlan& E, const vx_poly* P, int np, const vx_csf* S, bool bound = false) {
  const int k = S->k;
  E.k = k;
  for (int l = 0; l + 1 < k; l++) {
    const int m = k - l - 1;  // dimension of the trailing tuples left after depth l+1
    const int width = (l == k - 2) ? LEAF_W : 2;
    for (int p = 0; p < np; p++) {
      // leaf input written by a middle stage: entry-major, d + 1 + LEAF_PF_MAX
      // entry planes (the leaf reads up to entry d + LEAF_PF_MAX)
      const int64_t row = (k >= 3 && l == k - 2) ? P[p].degree + 1 + LEAF_PF_MAX
                          : (k == 3 && l == 0)   ? padded_entries(P[p].degree)
                                                 : ntup(m, P[p].degree);
      E.rows[l][p] = A.take<double>((size_t)S->n[l] * row * width + 4 * ROW_PAD * width) + 2 * ROW_PAD * width;
    }
  }
  E.R = stage1_blocking(S->n[0]);
  int64_t nmax = 0;
  for (int l = 0; l < k; l++) nmax = S->n[l] > nmax ? S->n[l] : nmax;
  for (int l = 0; l < k; l++) {
    const int64_t nparent = l == 0 ? 1 : S->n[l - 1];
    const int Z = bound ? 1 : l == k - 1 ? (S->n[k - 1] <= LEAF_ONE_NODES ? 1 : LEAF_R) : (l == 0 ? E.R : 64);
    const int pack = k == 3 && l == 1 && (bound || (S->n[1] >= PACK_MIN_NODES && nmax > SMALL_LEVEL_NODES));
    plan_segments(A, E.seg[l], nparent, S->n[l], Z, pack);
  }
}

size_t eval_workspace_bytes(const vx_poly* P, int np, const vx_csf* S) {
  Arena A;
  EvalPlan E;
  plan_eval(A, E, P, np, S);
  return A.off + prepared_bytes(P, np) + 512;
}

size_t eval_level_bytes(const vx_poly* P, int np, const vx_csf* S) {
  Arena A;
  EvalPlan E;
  plan_eval(A, E, P, np, S);
  return A.off + 256;
}

size_t eval_level_bytes_bound(const vx_poly* P, int np, const vx_csf* S) {
  Arena A;
  EvalPlan E;
  plan_eval(A, E, P, np, S, true);
  return A.off + 256;
}

static int launch_stage1(const Prepared& Q, int p0, int pn, const vx_csf* S, const double* dom, EvalPlan& E,
                         hipStream_t st) {
  const int k = S->k, m = k - 1;
  PolySet ps;
  memset(&ps, 0, sizeof ps);
  RowSet rs;
  memset(&rs, 0, sizeof rs);
  ps.np = pn;
  int nt_max = 0;
  double units = 0;
  const int width = 2;  // also the leaf input's LEAF_W when k = 2
  for (int i = 0; i < pn; i++) {
    const int p = p0 + i, d = Q.d[p];
    ps.p[i].packed = reinterpret_cast<const double2*>(Q.packed[p]);
    ps.p[i].ttab = Q.ttab[p];
    ps.p[i].lens2 = Q.lens2[p];
    ps.p[i].padlist = Q.padlist[p];
    ps.p[i].npad = k == 3 ? (int)padded_npad(d) : 0;
    ps.p[i].d = d;
    ps.p[i].nt = (int)ntup(m, d);
    nt_max = ps.p[i].nt > nt_max ? ps.p[i].nt : nt_max;
    rs.rows[i] = E.rows[0][p];
    rs.stride[i] = (k == 3 ? padded_entries(d) : ntup(m, d)) * width;
    rs.estride[i] = width;
    units += (double)(ntup(k, d) - ntup(m, d)) * (double)S->n[0];
  }
  const SegPlan& sp = E.seg[0];
  const int ny = (nt_max + 63) / 64 + 1;
  const int64_t maxseg = sp.maxseg > 0 ? sp.maxseg : 1;
  const int64_t items = maxseg * ny * pn, chunk = ny;
  const dim3 grid((unsigned)xcd_grid(items, chunk));
  const AxisGrid g = make_grid(dom, 0, S->level, E.mode[0]);
  const int4* sg = (const int4*)sp.seg;
  const int64_t* ns = (const int64_t*)sp.nseg;
  const int pr = prof_start("k_stage1", units, st);
  switch (E.R) {
    case 1: hipLaunchKernelGGL(k_stage1<1>, grid, dim3(64), 0, st, ps, m, S->idx[0], sg, ns, g, rs, width, maxseg, ny, chunk, items); break;
    case 2: hipLaunchKernelGGL(k_stage1<2>, grid, dim3(64), 0, st, ps, m, S->idx[0], sg, ns, g, rs, width, maxseg, ny, chunk, items); break;
    case 4: hipLaunchKernelGGL(k_stage1<4>, grid, dim3(64), 0, st, ps, m, S->idx[0], sg, ns, g, rs, width, maxseg, ny, chunk, items); break;
    default: hipLaunchKernelGGL(k_stage1<8>, grid, dim3(64), 0, st, ps, m, S->idx[0], sg, ns, g, rs, width, maxseg, ny, chunk, items); break;
  }
  VX_CHECK_LAUNCH("k_stage1");
  prof_stop(pr, st);
  return VX_OK;
}

static int launch_narrow(const Prepared& Q, int p0, int pn, int l, const vx_csf* S, const double* dom, EvalPlan& E,
                         hipStream_t st) {
  const int k = S->k;
  const int m_in = k - l, m_out = k - l - 1;
  const int width = (l == k - 2) ? LEAF_W : 2;
  PolySet ps;
  memset(&ps, 0, sizeof ps);
  RowSet in, out;
  memset(&in, 0, sizeof in);
  memset(&out, 0, sizeof out);
  SplitSet ss;
  memset(&ss, 0, sizeof ss);
  const int64_t est_waves = (S->n[l] + 63) / 64 + S->n[l - 1];
  int groups = (int)((NARROW_TARGET_WAVES + est_waves - 1) / est_waves);
  // padded rows (k = 3) split in the kernel, down to one chain per split;
  // the other layouts take a table of at most SPLIT_MAX splits
  const int gcap = k == 3 ? Q.dmax + 1 : SPLIT_MAX;
  groups = groups < 1 ? 1 : (groups > gcap ? gcap : groups);
  int gmax = 1;
  double units = 0;
  ps.np = pn;
  for (int i = 0; i < pn; i++) {
    const int p = p0 + i, d = Q.d[p];
    ps.p[i].lens2 = Q.lens2[p];
    ps.p[i].d = d;
    in.rows[i] = E.rows[l - 1][p];
    in.stride[i] = (k == 3 ? padded_entries(d) : ntup(m_in, d)) * 2;
    out.rows[i] = E.rows[l][p];
    const bool to_leaf = l == k - 2;
    out.stride[i] = to_leaf ? LEAF_W : ntup(m_out, d) * width;
    out.estride[i] = to_leaf ? LEAF_W * S->n[l] : width;
    if (k == 3) {
      gmax = groups;
    } else {
      ss.s[i] = chain_split(m_out, d, groups);
      gmax = ss.s[i].n > gmax ? ss.s[i].n : gmax;
    }
    units += (double)(ntup(m_in, d) - ntup(m_out, d)) * (double)S->n[l];
  }
  const SegPlan& sp = E.seg[l];
  const int64_t items = sp.maxseg * gmax * pn;
  dim3 grid((unsigned)xcd_grid(items, NARROW_XCD_CHUNK));
  const AxisGrid g = make_grid(dom, l, S->level, E.mode[l]);
  const int pr = prof_start("k_narrow", units, st);
  if (k == 3 && sp.pack) {
    TailLists tl;
    for (int c = 0; c < 2; c++) {
      tl.node[c] = sp.tnode[c];
      tl.par[c] = sp.tpar[c];
    }
    hipLaunchKernelGGL(k_narrow_mixed, grid, dim3(64), 0, st, ps, in, S->idx[l], (const int4*)sp.seg,
                       (const int64_t*)sp.nfull, (const int64_t*)sp.nseg, tl, g, out, width, sp.maxseg, gmax, items);
  } else if (k == 3) {
    hipLaunchKernelGGL((k_narrow<true, true>), grid, dim3(64), 0, st, ps, in, ss, S->idx[l], (const int4*)sp.seg,
                       (const int64_t*)sp.nseg, g, out, width, sp.maxseg, gmax, items);
  }
  else if (m_out == 1)
    hipLaunchKernelGGL((k_narrow<true, false>), grid, dim3(64), 0, st, ps, in, ss, S->idx[l], (const int4*)sp.seg,
                       (const int64_t*)sp.nseg, g, out, width, sp.maxseg, gmax, items);
  else
    hipLaunchKernelGGL((k_narrow<false, false>), grid, dim3(64), 0, st, ps, in, ss, S->idx[l], (const int4*)sp.seg,
                       (const int64_t*)sp.nseg, g, out, width, sp.maxseg, gmax, items);
  VX_CHECK_LAUNCH("k_narrow");
  prof_stop(pr, st);
  return VX_OK;
}

static int launch_leaf(const Prepared& Q, int p0, int pn, const vx_csf* S, const double* dom, EvalPlan& E,
                       double* lo, double* hi, uint8_t* keep, hipStream_t st, uint8_t* alive) {
  const int k = S->k;
  const int64_t nleaf = S->n[k - 1];
  PolySet ps;
  memset(&ps, 0, sizeof ps);
  RowSet rs;
  memset(&rs, 0, sizeof rs);
  ps.np = pn;
  double units = 0;
  for (int i = 0; i < pn; i++) {
    const int p = p0 + i, d = Q.d[p];
    ps.p[i].d = d;
    rs.rows[i] = k == 1 ? Q.packed[p] : E.rows[k - 2][p];
    rs.stride[i] = k == 1 ? 0 : (k == 2 ? LEAF_W * (int64_t)(d + 1) : LEAF_W);
    rs.estride[i] = k >= 3 ? LEAF_W * S->n[k - 2] : LEAF_W;
    units += (double)d * (double)nleaf;
  }
  const SegPlan& sp = E.seg[k - 1];
  const AxisGrid g = make_grid(dom, k - 1, S->level, E.mode[k - 1]);
  double* lo_p = lo + (int64_t)p0 * nleaf;
  double* hi_p = hi + (int64_t)p0 * nleaf;
  const int4* sg = (const int4*)sp.seg;
  const int64_t* ns = (const int64_t*)sp.nseg;
  const int first = p0 == 0 ? 1 : 0;
  const int pr = prof_start("k_leaf", units, st);
  const dim3 grid1((unsigned)((sp.maxseg + 255) / 256));
  if (sp.Z == 1) {  // one box per lane (the segments were built with Z = 1)
    int p2 = 1;
    while (p2 < pn) p2 <<= 1;
    const dim3 grid((unsigned)((sp.maxseg * p2 + 255) / 256));
    hipLaunchKernelGGL((k_leaf<true, 8, 1>), grid, dim3(256), 0, st, ps, rs, sg, ns, S->idx[k - 1], nleaf, g, lo_p,
                       hi_p, keep, first, p2, alive);
  } else if (nleaf <= LEAF_SPLIT_NODES && pn > 1) {
    int p2 = 1;
    while (p2 < pn) p2 <<= 1;
    const int64_t threads = sp.maxseg * p2;
    hipLaunchKernelGGL((k_leaf<true, 8, LEAF_R>), dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st, ps, rs,
                       sg, ns, S->idx[k - 1], nleaf, g, lo_p, hi_p, keep, first, p2, alive);
  } else if (nleaf <= LEAF_SPLIT_NODES) {
    hipLaunchKernelGGL((k_leaf<false, 8, LEAF_R>), grid1, dim3(256), 0, st, ps, rs, sg, ns, S->idx[k - 1], nleaf, g,
                       lo_p, hi_p, keep, first, 1, alive);
  } else {
    hipLaunchKernelGGL((k_leaf<false, 4, LEAF_R>), grid1, dim3(256), 0, st, ps, rs, sg, ns, S->idx[k - 1], nleaf, g,
                       lo_p, hi_p, keep, first, 1, alive);
  }
  VX_CHECK_LAUNCH("k_leaf");
  prof_stop(pr, st);
  return VX_OK;
}

int eval_level_prepared(const Prepared& Q, const vx_csf* S, const double* dom, double* lo, double* hi, uint8_t* keep,
                        void* ws, size_t ws_bytes, hipStream_t st, const vx_poly* P, int centre,
                        const int* axis_modes, uint8_t* alive) {
  const int k = S->k;
  const int64_t nleaf = S->n[k - 1];
  if (nleaf == 0) return VX_OK;
  Arena A;
  A.base = reinterpret_cast<char*>(ws);
  A.size = ws_bytes;
  EvalPlan E;
  plan_eval(A, E, P, Q.np, S);
  for (int l = 0; l < k; l++) E.mode[l] = axis_modes ? axis_modes[l] : centre;
  if (A.overflow)
    VX_FAIL(VX_ECAPACITY, "interval_eval_level: workspace of %zu bytes is too small (%zu needed)", ws_bytes,
            A.off + 256);
  int rc;
  int64_t nmax = 0;
  for (int l = 0; l < k; l++) nmax = S->n[l] > nmax ? S->n[l] : nmax;
  SegJob J;
  memset(&J, 0, sizeof J);
  for (int l = 0; l < k; l++) {
    const SegPlan& sp = E.seg[l];
    J.ptr[l] = l == 0 ? nullptr : S->ptr[l - 1];
    J.labels[l] = S->idx[l];
    J.g[l] = make_grid(dom, l, S->level, E.mode[l]);
    J.Z[l] = sp.Z;
    J.nparent[l] = sp.nparent;
    J.nchild[l] = sp.nchild;
    J.cnt[l] = sp.cnt;
    J.bounds[l] = sp.bounds;
    J.off[l] = sp.off;
    J.seg[l] = sp.seg;
    J.nseg[l] = sp.nseg;
  }
  J.pl = -1;
  if (!keep || k < 2) alive = nullptr;
  J.alive = alive;
  for (int l = 0; l < k; l++)
    if (E.seg[l].pack) {
      const SegPlan& sp = E.seg[l];
      J.pl = l;
      J.nfull = sp.nfull;
      for (int c = 0; c < 2; c++) {
        J.tcnt[c] = sp.tcnt[c];
        J.toff[c] = sp.toff[c];
        J.ttot[c] = sp.ttot[c];
        J.tnode[c] = sp.tnode[c];
        J.tpar[c] = sp.tpar[c];
      }
    }
  if (nmax <= SMALL_LEVEL_NODES && J.pl < 0) {
    hipLaunchKernelGGL(k_segments_small, dim3(1), dim3(SMALL_THREADS), 0, st, k, J);
    VX_CHECK_LAUNCH("k_segments_small");
  } else {
    const DepthBlocks D = depth_blocks(J.nparent, k, 256);
    const dim3 grid(D.blocks());
    hipLaunchKernelGGL(k_seg_count_all, grid, dim3(256), 0, st, D, J);
    VX_CHECK_LAUNCH("k_seg_count_all");
    MultiScan<int64_t, int64_t> M;
    memset(&M, 0, sizeof M);
    int na = 0;
    for (int l = 0; l < k; l++, na++) {
      M.in[na] = E.seg[l].cnt;
      M.out[na] = E.seg[l].off;
      M.total[na] = E.seg[l].pack ? E.seg[l].nfull : E.seg[l].nseg;
      M.tiles[na] = E.seg[l].tiles;
      M.n[na] = E.seg[l].nparent;
    }
    if (J.pl >= 0)
      for (int c = 0; c < 2; c++, na++) {
        const SegPlan& sp = E.seg[J.pl];
        M.in[na] = sp.tcnt[c];
        M.out[na] = sp.toff[c];
        M.total[na] = sp.ttot[c];
        M.tiles[na] = sp.ttiles[c];
        M.n[na] = sp.nparent;
      }
    multi_scan(M, na, st);
    VX_CHECK_LAUNCH("segment scans");
    hipLaunchKernelGGL(k_seg_write_all, grid, dim3(256), 0, st, D, J);
    VX_CHECK_LAUNCH("k_seg_write_all");
  }
  for (int p0 = 0; p0 < Q.np; p0 += PMAX) {
    const int pn = Q.np - p0 < PMAX ? Q.np - p0 : PMAX;
    if (k >= 2 && (rc = launch_stage1(Q, p0, pn, S, dom, E, st))) return rc;
    for (int l = 1; l + 1 < k; l++)
      if ((rc = launch_narrow(Q, p0, pn, l, S, dom, E, st))) return rc;
    if ((rc = launch_leaf(Q, p0, pn, S, dom, E, lo, hi, keep, st, p0 + pn == Q.np ? alive : nullptr))) return rc;
  }
  return VX_OK;
}

int eval_level_impl(const vx_poly* P, int np, const vx_csf* S, const double* dom, double* lo, double* hi,
                    uint8_t* keep, void* ws, size_t ws_bytes, hipStream_t st, int centre) {
  if (S->n[S->k - 1] == 0) return VX_OK;
  const size_t qb = prepared_bytes(P, np);
  if (qb > ws_bytes) VX_FAIL(VX_ECAPACITY, "interval_eval_level: workspace too small");
  Prepared Q;
  int rc;
  if ((rc = prepare_polys(P, np, ws, qb, &Q, st))) return rc;
  return eval_level_prepared(Q, S, dom, lo, hi, keep, reinterpret_cast<char*>(ws) + qb, ws_bytes - qb, st, P,
                             centre);
}

// Batched persistent subdivision of many systems (same translation unit: it
// reuses the device functions above).
#include "batch.inc"

}  // namespace vx
