// Point evaluation with gradients, the coefficient adjoint on a CSF grid of
// cell centres, and Newton projection (Moroz, arXiv 2406.09857, Sec. 3.2:
// Newton steps in the span of the gradients when a system has fewer equations
// than unknowns; the Taylor/mean-value form uses the gradient on a box).
//
// Arithmetic is ordinary round-to-nearest FP64.  Values use no fused
// multiply-add and follow the same nested Horner order as the interval path
// (x1 innermost, descending exponents), so F(x) is bit-identical to a plain
// nested Horner evaluation; derivatives are carried forward-mode along the
// same chains (d(v*x + c)/dx = (dv/dx)*x + v), each step one fused
// multiply-add (one rounding instead of two), the same in the per-point and
// the grid evaluation, so their Jacobians agree bit for bit.
#include <hip/hip_runtime.h>
#include <string.h>

#include "common.hpp"
#include "eval.hpp"
#include "grad.hpp"
#include "scan.hpp"

namespace vx {

__host__ __device__ inline int64_t gbinom(int n, int r) {
  if (r < 0 || n < r) return 0;
  int64_t v = 1;
  for (int i = 1; i <= r; i++) v = v * (n - r + i) / i;
  return v;
}

// O_m position (consumption order: for t' in O_{m-1}: for e desc).
__device__ inline int64_t g_opos(const int* t, int m, int d) {
  int64_t pos = 0;
  int sigma = 0;
  for (int j = m; j >= 1; j--) {
    sigma += t[j - 1];
    pos += gbinom(d - sigma + j - 1, j);
  }
  return pos;
}

// Graded order of m-tuples: by total degree, then lexicographic (t0, t1, ...).
__device__ inline int64_t g_rank(const int* t, int m) {
  if (m == 0) return 0;
  int g = 0;
  for (int i = 0; i < m; i++) g += t[i];
  int64_t r = gbinom(g + m - 1, m);
  int pre = 0;
  for (int i = 0; i + 1 < m; i++) {
    for (int v = 0; v < t[i]; v++) r += gbinom(g - pre - v + (m - 1 - i) - 1, (m - 1 - i) - 1);
    pre += t[i];
  }
  return r;
}

__device__ inline void g_unrank(int64_t r, int m, int* t) {
  if (m == 0) return;
  int g = 0;
  while (gbinom(g + 1 + m - 1, m) <= r) g++;
  r -= gbinom(g + m - 1, m);
  int pre = 0;
  for (int i = 0; i + 1 < m; i++) {
    int v = 0;
    while (true) {
      const int64_t c = gbinom(g - pre - v + (m - 1 - i) - 1, (m - 1 - i) - 1);
      if (r < c) break;
      r -= c;
      v++;
    }
    t[i] = v;
    pre += v;
  }
  t[m - 1] = g - pre;
}

// Cell centre of `label` at `level` on [dlo, dhi], round to nearest (exact
// on dyadic domains).
__device__ __forceinline__ double centre(double dlo, double dhi, int level, int32_t label) {
  return dlo + ldexp((double)(2 * (int64_t)label + 1) * (dhi - dlo), -(level + 1));
}

// ---------------------------------------------------------------------------
// Nested coefficient stream: chains in O_{k-1} order of their trailing tuple,
// each chain c[e1 = d-|t| .. 0, t] front-padded with zeros to a multiple of
// SG entries (a group of SG scalar loads per step of the chain loop; groups
// of 4 waste fewer padding steps on short chains than groups of 8 and keep
// the loads ahead of the arithmetic: 3 % faster Newton steps on the curve).
// ---------------------------------------------------------------------------
constexpr int SG = 4;

__global__ void k_stream_len(int k, int d, int side, int64_t* __restrict__ plen) {
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t total = 1;
  for (int i = 1; i < k; i++) total *= side;
  if (f >= total) return;  // enumerate trailing tuples t (k-1 coordinates)
  int t[VX_KMAX] = {0, 0, 0, 0};
  int64_t q = f;
  for (int i = k - 2; i >= 0; i--) { t[i] = (int)(q % side); q /= side; }
  int deg = 0;
  for (int i = 0; i + 1 < k; i++) deg += t[i];
  if (deg > d) return;
  const int64_t L = d - deg + 1;
  plen[k >= 2 ? g_opos(t, k - 1, d) : 0] = (L + SG - 1) / SG * SG;
}

__global__ void k_stream_fill(int k, int d, int side, const double* __restrict__ c, const int64_t* __restrict__ start,
                              double* __restrict__ stream) {
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
  const int tdeg = deg - e[0];
  const int64_t ch = k >= 2 ? g_opos(e + 1, k - 1, d) : 0;
  const int64_t L = d - tdeg + 1;
  const int64_t pad = (L + SG - 1) / SG * SG - L;
  stream[start[ch] + pad + (d - tdeg - e[0])] = c[f];
}

struct I64Load {
  const int64_t* a;
  __device__ int64_t operator()(int64_t i) const { return a[i]; }
};

// ---------------------------------------------------------------------------
// Per-point evaluation: lanes are points, the stream is wave-uniform.
// ---------------------------------------------------------------------------
typedef __attribute__((address_space(4))) const double cdbl_t;

__device__ __forceinline__ int64_t after_d(double x) {
  int64_t z;
  asm volatile("s_mov_b64 %0, 0" : "=s"(z) : "s"(x));
  return z;
}

// Value and gradient of one polynomial at the lane's PP points (each
// coefficient load serves all of them; every point's arithmetic is the same,
// in the same order, whatever PP).  `grad` may be skipped (GRAD = false) for
// value-only evaluation.
template <int K, bool GRAD, int PP>
__device__ void point_eval(const cdbl_t* __restrict__ S, int d, const double (&x)[PP][VX_KMAX], double (&val)[PP],
                           double (&grad)[PP][VX_KMAX]) {
  // acc[q][s]: Horner accumulator of depth s (s = 0 is the x1 chain) of point q;
  // der[q][s][j]: its derivative with respect to x_j (j <= s).
  double acc[PP][K], der[PP][K][K];
#pragma unroll
  for (int q = 0; q < PP; q++)
#pragma unroll
    for (int s = 0; s < K; s++) {
      acc[q][s] = 0.0;
#pragma unroll
      for (int j = 0; j < K; j++) der[q][s][j] = 0.0;
    }
  double A[SG];
  int64_t g = 0;
#pragma unroll
  for (int e = 0; e < SG; e++) A[e] = S[e];
  // loops over the trailing tuple in O_{K-1} order (outermost variable first)
  int t[VX_KMAX] = {0, 0, 0, 0};
  auto chain = [&](int L) {  // one x1 chain of L entries, padded
    const int ng = (L + SG - 1) / SG;
#pragma unroll
    for (int q = 0; q < PP; q++) {
      acc[q][0] = 0.0;
      if (GRAD) der[q][0][0] = 0.0;
    }
    for (int gg = 0; gg < ng; gg++) {
      const int64_t z = after_d(A[0]);
      double B[SG];
#pragma unroll
      for (int e = 0; e < SG; e++) B[e] = S[(g + 1) * SG + z + e];
#pragma unroll
      for (int e = 0; e < SG; e++)
#pragma unroll
        for (int q = 0; q < PP; q++) {
          if (GRAD) der[q][0][0] = fma(der[q][0][0], x[q][0], acc[q][0]);
          acc[q][0] = acc[q][0] * x[q][0] + A[e];
        }
#pragma unroll
      for (int e = 0; e < SG; e++) A[e] = B[e];
      g++;
    }
  };
  // fold accumulator s-1 into s (Horner step in x_s)
  auto fold = [&](int s) {
#pragma unroll
    for (int q = 0; q < PP; q++) {
      if (GRAD) {
#pragma unroll
        for (int j = 0; j < K; j++) {
          if (j < s) der[q][s][j] = fma(der[q][s][j], x[q][s], der[q][s - 1][j]);
          else if (j == s) der[q][s][j] = fma(der[q][s][j], x[q][s], acc[q][s]);
        }
      }
      acc[q][s] = acc[q][s] * x[q][s] + acc[q][s - 1];
    }
  };
  auto reset = [&](int s) {
#pragma unroll
    for (int q = 0; q < PP; q++) {
      acc[q][s] = 0.0;
      if (GRAD) {
#pragma unroll
        for (int j = 0; j < K; j++) der[q][s][j] = 0.0;
      }
    }
  };
  if (K == 1) {
    chain(d + 1);
  } else if (K == 2) {
    for (t[0] = d; t[0] >= 0; t[0]--) {
      chain(d - t[0] + 1);
      fold(1);
    }
  } else if (K == 3) {
    for (int e3 = d; e3 >= 0; e3--) {
      reset(1);
      for (int e2 = d - e3; e2 >= 0; e2--) {
        chain(d - e2 - e3 + 1);
        fold(1);
      }
      fold(2);
    }
  } else {
    for (int e4 = d; e4 >= 0; e4--) {
      reset(2);
      for (int e3 = d - e4; e3 >= 0; e3--) {
        reset(1);
        for (int e2 = d - e3 - e4; e2 >= 0; e2--) {
          chain(d - e2 - e3 - e4 + 1);
          fold(1);
        }
        fold(2);
      }
      fold(3);
    }
  }
#pragma unroll
  for (int q = 0; q < PP; q++) {
    val[q] = acc[q][K - 1];
    if (GRAD) {
#pragma unroll
      for (int j = 0; j < K; j++) grad[q][j] = der[q][K - 1][j];
    }
  }
}

struct StreamSet {
  const double* s[PMAX_GRAD];
  int d[PMAX_GRAD];
};

// Points per lane of the per-point kernels (point q of the lane is point
// blockIdx.x * 64 * PPL + q * 64 + lane).
constexpr int PPL = 2;

template <int K, bool GRAD>
__global__ __launch_bounds__(64) void k_point_eval(StreamSet ss, int np, const double* __restrict__ x, int64_t n,
                                                   double* __restrict__ f, double* __restrict__ jac) {
  const int p = blockIdx.y;
  const int64_t i0 = (int64_t)blockIdx.x * 64 * PPL + threadIdx.x;
  double xi[PPL][VX_KMAX] = {};
#pragma unroll
  for (int q = 0; q < PPL; q++) {
    const int64_t i = i0 + q * 64;
#pragma unroll
    for (int j = 0; j < K; j++) xi[q][j] = i < n ? x[i * K + j] : 0.0;
  }
  double v[PPL], gr[PPL][VX_KMAX];
  point_eval<K, GRAD, PPL>((const cdbl_t*)ss.s[p], ss.d[p], xi, v, gr);
#pragma unroll
  for (int q = 0; q < PPL; q++) {
    const int64_t i = i0 + q * 64;
    if (i >= n) continue;
    f[p * n + i] = v[q];
    if (GRAD && jac) {
#pragma unroll
      for (int j = 0; j < K; j++) jac[(i * np + p) * K + j] = gr[q][j];
    }
  }
}

// Newton projection: x <- x - J^T (J J^T)^{-1} F, J the np x K Jacobian
// (minimum-norm step in the span of the gradients).
// Newton step of one point from its values F and Jacobian J (np x K).
template <int K>
__device__ __forceinline__ void newton_update(int np, const double (&F)[PMAX_GRAD],
                                              const double (&J)[PMAX_GRAD][VX_KMAX], double (&xi)[VX_KMAX]) {
  // M = J J^T (np x np), solve M y = F by elimination with partial pivoting
  double M[PMAX_GRAD][PMAX_GRAD + 1];
  for (int a = 0; a < np; a++) {
    for (int b = 0; b < np; b++) {
      double s = 0.0;
#pragma unroll
      for (int j = 0; j < K; j++) s += J[a][j] * J[b][j];
      M[a][b] = s;
    }
    M[a][np] = F[a];
  }
  bool ok = true;
  for (int c = 0; c < np && ok; c++) {
    int piv = c;
    for (int r = c + 1; r < np; r++)
      if (fabs(M[r][c]) > fabs(M[piv][c])) piv = r;
    if (!(fabs(M[piv][c]) > 1e-300)) { ok = false; break; }
    if (piv != c)
      for (int q = 0; q <= np; q++) {
        const double tmp = M[c][q];
        M[c][q] = M[piv][q];
        M[piv][q] = tmp;
      }
    for (int r = c + 1; r < np; r++) {
      const double fct = M[r][c] / M[c][c];
      for (int q = c; q <= np; q++) M[r][q] -= fct * M[c][q];
    }
  }
  if (ok) {
    double y[PMAX_GRAD];
    for (int r = np - 1; r >= 0; r--) {
      double s = M[r][np];
      for (int q = r + 1; q < np; q++) s -= M[r][q] * y[q];
      y[r] = s / M[r][r];
    }
#pragma unroll
    for (int j = 0; j < K; j++) {
      double s = 0.0;
      for (int p = 0; p < np; p++) s += J[p][j] * y[p];
      xi[j] -= s;
    }
  }
}

// `steps` Newton steps on the lane's points.  f0, j0 (may be null): F and J
// at the starting points, already evaluated (f0[p * n + i],
// j0[(i * np + p) * K + j]); the first evaluation is then taken from them.
// F at the final points needs no derivatives: the host evaluates it with
// k_point_eval<K, false> after this kernel.
template <int K>
__global__ __launch_bounds__(64) void k_newton(StreamSet ss, int np, double* __restrict__ x, int64_t n, int steps,
                                               const double* __restrict__ f0, const double* __restrict__ j0) {
  const int64_t i0 = (int64_t)blockIdx.x * 64 * PPL + threadIdx.x;
  double xi[PPL][VX_KMAX] = {};
#pragma unroll
  for (int q = 0; q < PPL; q++) {
    const int64_t i = i0 + q * 64;
#pragma unroll
    for (int j = 0; j < K; j++) xi[q][j] = i < n ? x[i * K + j] : 0.0;
  }
  double F[PPL][PMAX_GRAD], J[PPL][PMAX_GRAD][VX_KMAX];
  for (int it = 0; it < steps; it++) {
    for (int p = 0; p < np; p++) {
      double v[PPL], gr[PPL][VX_KMAX];
      if (it == 0 && f0) {
#pragma unroll
        for (int q = 0; q < PPL; q++) {
          const int64_t i = i0 + q * 64 < n ? i0 + q * 64 : n - 1;
          v[q] = f0[p * n + i];
#pragma unroll
          for (int j = 0; j < K; j++) gr[q][j] = j0[(i * np + p) * K + j];
        }
      } else {
        point_eval<K, true, PPL>((const cdbl_t*)ss.s[p], ss.d[p], xi, v, gr);
      }
#pragma unroll
      for (int q = 0; q < PPL; q++) {
        F[q][p] = v[q];
#pragma unroll
        for (int j = 0; j < K; j++) J[q][p][j] = gr[q][j];
      }
    }
#pragma unroll
    for (int q = 0; q < PPL; q++) newton_update<K>(np, F[q], J[q], xi[q]);
  }
#pragma unroll
  for (int q = 0; q < PPL; q++) {
    const int64_t i = i0 + q * 64;
    if (i >= n) continue;
#pragma unroll
    for (int j = 0; j < K; j++) x[i * K + j] = xi[q][j];
  }
}

// Centres of the leaves of a CSF (n x k, RN).
__global__ void k_csf_centres(int k, int level, const int32_t* i0, const int32_t* i1, const int32_t* i2,
                              const int32_t* i3, const int32_t* p0, const int32_t* p1, const int32_t* p2,
                              int64_t n0, int64_t n1, int64_t n2, int64_t nleaf, AxisDom dom,
                              double* __restrict__ x) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nleaf) return;
  const int32_t* idx[4] = {i0, i1, i2, i3};
  const int32_t* ptr[3] = {p0, p1, p2};
  const int64_t nn[3] = {n0, n1, n2};
  int64_t node = b;
  for (int l = k - 1; l >= 0; l--) {
    x[b * k + l] = centre(dom.lo[l], dom.hi[l], level, idx[l][node]);
    if (l > 0) {  // parent: last q with ptr[l-1][q] <= node
      int64_t lo = 0, hi = nn[l - 1];
      while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (ptr[l - 1][mid] <= node) lo = mid; else hi = mid;
      }
      node = lo;
    }
  }
}

// ---------------------------------------------------------------------------
// Coefficient adjoint on a CSF grid of centres: the transpose of the
// amortized evaluation.  Depth by depth from the leaves, every parent row is
//   out[(e, t)] = sum_{children q} x(q)^e * in_q[t]
// (graded order of tuples); the leaf input is gbar.  Each output entry is one
// lane summing over the children in order (deterministic).  Children come in
// chunks of ADJ_CHUNK: their powers x^0..x^d (repeated multiplication) and,
// where the input rows are short (stage_w entries each: 1 at the leaf depth,
// d + 1 one depth up), the rows themselves are staged in LDS with one
// coalesced load, so the sums read LDS only.  Dynamic LDS:
// ADJ_CHUNK (d + 1 + 1 + stage_w) doubles.
// ---------------------------------------------------------------------------
constexpr int ADJ_CHUNK = 32;
constexpr size_t ADJ_LDS_MAX = 64 * 1024;

__host__ __device__ inline size_t adjoint_lds_bytes(int d, int stage_w) {
  return sizeof(double) * (size_t)ADJ_CHUNK * (size_t)(d + 2 + stage_w);
}

__global__ __launch_bounds__(256) void k_adjoint_level(int d, int m_in, const int32_t* __restrict__ ptr,
                                                       int64_t nroot_children, const int32_t* __restrict__ labels,
                                                       double dlo, double dhi, int level,
                                                       const double* __restrict__ in, int64_t in_stride,
                                                       double* __restrict__ out, int64_t out_stride,
                                                       int64_t nout, int stage_w) {
  extern __shared__ double adj_lds[];
  const int W = d + 1;
  double* pw = adj_lds;                 // [ADJ_CHUNK][W]
  double* xs = pw + ADJ_CHUNK * W;      // [ADJ_CHUNK]
  double* ins = xs + ADJ_CHUNK;         // [ADJ_CHUNK][stage_w]
  const int64_t parent = blockIdx.x;
  const int64_t o = (int64_t)blockIdx.y * blockDim.x + threadIdx.x;
  const bool act = o < nout;
  // (e, t) of output rank o: closed forms for output tuples of dimension 1
  // (rank e), 2 (rank g (g + 1) / 2 + e, g = e + t1) and 3 (C(g + 2, 3)
  // tuples of lower degree, then e (g + 1) - e (e - 1) / 2 with a smaller
  // first coordinate, then t1), each estimate corrected in integers; the
  // generic walk above that
  int e = 0;
  int64_t tin = 0;
  if (act && m_in == 0) {
    e = (int)o;
  } else if (act && m_in == 1) {
    int64_t g = (int64_t)((sqrt(8.0 * (double)o + 1.0) - 1.0) * 0.5);
    while ((g + 1) * (g + 2) / 2 <= o) g++;
    while (g * (g + 1) / 2 > o) g--;
    e = (int)(o - g * (g + 1) / 2);
    tin = g - e;
  } else if (act && m_in == 2) {
    int64_t g = (int64_t)cbrt(6.0 * (double)o);
    while ((g + 1) * (g + 2) * (g + 3) / 6 <= o) g++;
    while (g > 0 && g * (g + 1) * (g + 2) / 6 > o) g--;
    const int64_t r = o - g * (g + 1) * (g + 2) / 6;
    const double a = 2.0 * (double)g + 3.0;
    const double disc = a * a - 8.0 * (double)r;
    int64_t v = (int64_t)((a - sqrt(disc > 0.0 ? disc : 0.0)) * 0.5);
    auto before = [&](int64_t x) { return x * (g + 1) - x * (x - 1) / 2; };
    while (v < g && before(v + 1) <= r) v++;
    while (v > 0 && before(v) > r) v--;
    const int64_t t1 = r - before(v), t2 = g - v - t1, gt = t1 + t2;
    e = (int)v;
    tin = gt * (gt + 1) / 2 + t1;
  } else if (act) {
    int tt[VX_KMAX] = {0, 0, 0, 0};
    g_unrank(o, m_in + 1, tt);
    e = tt[0];
    tin = g_rank(tt + 1, m_in);
  }
  const int64_t b = ptr ? ptr[parent] : 0, en = ptr ? ptr[parent + 1] : nroot_children;
  double acc = 0.0;
  for (int64_t c0 = b; c0 < en; c0 += ADJ_CHUNK) {
    const int cn = (int)(en - c0 < ADJ_CHUNK ? en - c0 : ADJ_CHUNK);
    __syncthreads();
    if (threadIdx.x < cn) xs[threadIdx.x] = centre(dlo, dhi, level, labels[c0 + threadIdx.x]);
    // rows of consecutive children are consecutive (in_stride == stage_w)
    for (int i = threadIdx.x; i < cn * stage_w; i += blockDim.x) ins[i] = in[c0 * in_stride + i];
    __syncthreads();
    // powers x^0..x^d of every child in the chunk, by repeated multiplication
    // (x held in a register: the table's stores could alias xs)
    for (int q = threadIdx.x; q < cn; q += blockDim.x) {
      const double xq = xs[q];
      double p = 1.0;
      for (int j = 0; j <= d; j++) {
        pw[q * W + j] = p;
        p = p * xq;
      }
    }
    __syncthreads();
    if (act) {
      if (stage_w)
        for (int q = 0; q < cn; q++) acc += pw[q * W + e] * ins[q * stage_w + tin];
      else
        for (int q = 0; q < cn; q++) acc += pw[q * W + e] * in[(c0 + q) * in_stride + tin];
    }
  }
  if (act) out[parent * out_stride + o] = acc;
}

// Scatter the root row (graded order, dimension k) into the dense cube.
__global__ void k_adjoint_scatter(int k, int d, int side, const double* __restrict__ row, int64_t nrow,
                                  double* __restrict__ cube) {
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= nrow) return;
  int t[VX_KMAX] = {0, 0, 0, 0};
  g_unrank(o, k, t);
  int64_t f = 0;
  for (int i = 0; i < k; i++) f = f * side + t[i];
  cube[f] = row[o];
}

// ---------------------------------------------------------------------------
// Amortized point evaluation on a CSF grid of centres (Algorithm 2 with
// points for boxes, round to nearest).  When the points are the centres of
// the leaves of a CSF, every partial evaluation of the nested Horner above
// is shared by all points below one node, exactly as the interval path
// shares it between boxes: the x1 chains run once per depth-1 node, the x2
// chains once per depth-2 node, and so on (Theorem 1's count with points).
// A stage runs, for every node, the very instructions that the per-point
// evaluation runs for each point below it -- acc <- acc*x + c, the earlier
// variables' derivatives der_j <- fma(der_j, x, c_j) and the stage's own
// der_s <- fma(der_s, x, acc) (old acc), starting from zero -- so values and
// derivatives are bit-identical to k_point_eval.
//
// Rows.  Node q of depth l (l = 1..k-1) holds, for every trailing tuple of
// dimension k-l in O_{k-l} order, the partial evaluation and (with
// derivatives) its derivatives with respect to x_1..x_l: l+1 planes of
// `cstride` doubles.  The root row is the padded coefficient stream (one
// plane).  Stage l walks chains of its parent's row: output entry j is the
// chain of clen[j] entries starting at cstart[j].
// ---------------------------------------------------------------------------

// Chain table of a stage whose output tuples have dimension m_out (input
// rows in O_{m_out+1} order, unpadded): one thread per output tuple.
__global__ void k_grid_chains(int m_out, int d, int64_t nch, int64_t* __restrict__ cstart,
                              int64_t* __restrict__ clen) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nch) return;
  int t[VX_KMAX + 1] = {0, 0, 0, 0, 0};
  g_unrank(r, m_out, t + 1);
  int deg = 0;
  for (int i = 1; i <= m_out; i++) deg += t[i];
  t[0] = d - deg;  // first entry of the chain: the largest exponent of the stage's variable
  const int64_t pos = m_out ? g_opos(t + 1, m_out, d) : 0;
  cstart[pos] = g_opos(t, m_out + 1, d);
  clen[pos] = d - deg + 1;
}

// Parent index of every node of a depth (one thread per parent).
__global__ void k_grid_parents(const int32_t* __restrict__ ptr, int64_t nparent, int32_t* __restrict__ parent) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nparent) return;
  for (int64_t q = ptr[p]; q < ptr[p + 1]; q++) parent[q] = (int32_t)p;
}

// Stage L (1..k) for one polynomial: lane = node of depth L, blockIdx.y =
// chain group (the groups cut the parent row into runs of about equal
// length at chain boundaries, found by a binary search on cstart).  The
// lanes of a wave are consecutive nodes, mostly children of one parent, so
// their row loads mostly hit one address.  GRAD = false carries the value
// only.  The last stage (a single chain) writes f and jac.
template <int L, bool GRAD>
__global__ __launch_bounds__(256) void k_grid_stage(const double* __restrict__ in, int64_t in_stride,
                                                    int64_t in_cstride, const int32_t* __restrict__ parent,
                                                    const int32_t* __restrict__ labels, double dlo, double dhi,
                                                    int level, const int64_t* __restrict__ cstart,
                                                    const int64_t* __restrict__ clen, int64_t nch, int ngroup,
                                                    int64_t nnode, double* __restrict__ out, int64_t out_stride,
                                                    int64_t out_cstride, double* __restrict__ f,
                                                    double* __restrict__ jac, int np, int p, int k) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nnode) return;
  // chain group: [first chain starting at or after total*g/G, same for g+1)
  const int64_t total = cstart[nch - 1] + clen[nch - 1];
  auto first_at = [&](int g) -> int64_t {
    if (g >= ngroup) return nch;
    const int64_t target = (total * g + ngroup - 1) / ngroup;
    int64_t lo = 0, hi = nch;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (cstart[mid] >= target) hi = mid; else lo = mid + 1;
    }
    return lo;
  };
  const int64_t j0 = first_at(blockIdx.y), j1 = first_at(blockIdx.y + 1);
  const int64_t par = parent ? parent[q] : 0;
  const double x = centre(dlo, dhi, level, labels[q]);
  const double* row = in + par * in_stride;
  constexpr int NIN = GRAD ? L : 1;  // input planes: value, d/dx_1 .. d/dx_{L-1}
  for (int64_t j = j0; j < j1; j++) {
    const double* c = row + cstart[j];
    const int64_t len = clen[j];
    double acc = 0.0;
    double der[L] = {};
#pragma unroll 4
    for (int64_t e = 0; e < len; e++) {
      double cin[NIN];
#pragma unroll
      for (int i = 0; i < NIN; i++) cin[i] = c[i * in_cstride + e];
      if (GRAD) {
#pragma unroll
        for (int i = 1; i < NIN; i++) der[i - 1] = fma(der[i - 1], x, cin[i]);
        der[L - 1] = fma(der[L - 1], x, acc);
      }
      acc = acc * x + cin[0];
    }
    if (out) {
      double* o = out + q * out_stride + j;
      o[0] = acc;
      if (GRAD) {
#pragma unroll
        for (int i = 0; i < L; i++) o[(i + 1) * out_cstride] = der[i];
      }
    } else {
      f[p * nnode + q] = acc;
      if (GRAD && jac) {
#pragma unroll
        for (int i = 0; i < L; i++) jac[(q * np + p) * k + i] = der[i];
      }
    }
  }
}

// Flag (bit 0) any point that is not, bit for bit, the centre of its leaf
// as csf_centres writes it.
__global__ void k_check_centres(int k, int level, const int32_t* i0, const int32_t* i1, const int32_t* i2,
                                const int32_t* i3, const int32_t* p0, const int32_t* p1, const int32_t* p2,
                                int64_t n0, int64_t n1, int64_t n2, int64_t nleaf, AxisDom dom,
                                const double* __restrict__ x, unsigned int* __restrict__ bad) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nleaf) return;
  const int32_t* idx[4] = {i0, i1, i2, i3};
  const int32_t* ptr[3] = {p0, p1, p2};
  const int64_t nn[3] = {n0, n1, n2};
  int64_t node = b;
  bool ok = true;
  for (int l = k - 1; l >= 0; l--) {
    const double c = centre(dom.lo[l], dom.hi[l], level, idx[l][node]);
    ok = ok && __double_as_longlong(c) == __double_as_longlong(x[b * k + l]);
    if (l > 0) {
      int64_t lo = 0, hi = nn[l - 1];
      while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (ptr[l - 1][mid] <= node) lo = mid; else hi = mid;
      }
      node = lo;
    }
  }
  if (!ok) atomicOr(bad, 1u);
}

__global__ void k_zero_u32(unsigned int* p) {
  if (threadIdx.x == 0) *p = 0u;
}

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------
struct GradPlan {
  double* stream[PMAX_GRAD] = {};
  int64_t* plen[PMAX_GRAD] = {};
  int64_t* start[PMAX_GRAD] = {};
  int64_t* tiles = nullptr;
  int64_t slen[PMAX_GRAD] = {};
};

static int64_t stream_chains(int k, int d) { return k >= 2 ? gbinom(d + k - 1, k - 1) : 1; }

static int64_t stream_len_host(int k, int d) {
  // sum over trailing tuples of SG*ceil((d-|t|+1)/SG): tuples of degree g: C(g+k-2, k-2)
  int64_t s = 0;
  for (int g = 0; g <= d; g++) {
    const int64_t cnt = k >= 2 ? gbinom(g + k - 2, k - 2) : (g == 0 ? 1 : 0);
    s += cnt * ((int64_t)(d - g + 1 + SG - 1) / SG * SG);
  }
  return s;
}

static void plan_grad(Arena& A, GradPlan& G, const vx_poly* P, int np) {
  int64_t maxch = 1;
  for (int p = 0; p < np; p++) {
    const int k = P[p].k, d = P[p].degree;
    G.slen[p] = stream_len_host(k, d);
    G.stream[p] = A.take<double>(G.slen[p] + 2 * SG);
    const int64_t nch = stream_chains(k, d);
    G.plen[p] = A.take<int64_t>(nch + 1);
    G.start[p] = A.take<int64_t>(nch + 1);
    maxch = nch > maxch ? nch : maxch;
  }
  G.tiles = A.take<int64_t>(scan_tiles(maxch));
}

static int build_streams(GradPlan& G, const vx_poly* P, int np, hipStream_t st) {
  for (int p = 0; p < np; p++) {
    const int k = P[p].k, d = P[p].degree, side = P[p].side;
    const int64_t nch = stream_chains(k, d);
    int64_t tcube = 1;
    for (int i = 1; i < k; i++) tcube *= side;
    hipLaunchKernelGGL(k_stream_len, dim3((unsigned)((tcube + 255) / 256)), dim3(256), 0, st, k, d, side, G.plen[p]);
    VX_CHECK_LAUNCH("k_stream_len");
    scan_exclusive(I64Load{G.plen[p]}, (const int64_t*)nullptr, nch, G.start[p], (int64_t*)nullptr, G.tiles, st);
    VX_CHECK_LAUNCH("stream scan");
    VX_HIP(hipMemsetAsync(G.stream[p], 0, sizeof(double) * (G.slen[p] + 2 * SG), st));
    int64_t cube = tcube * side;
    hipLaunchKernelGGL(k_stream_fill, dim3((unsigned)((cube + 255) / 256)), dim3(256), 0, st, k, d, side, P[p].c_lo,
                       (const int64_t*)G.start[p], G.stream[p]);
    VX_CHECK_LAUNCH("k_stream_fill");
  }
  return VX_OK;
}

// Workspace of the amortized forward on a grid: the rows of depths 1..k-1
// (sized for the largest degree; reused polynomial after polynomial), the
// parent index of every node below depth 1, the chain tables of stages
// 2..k, and the centre-check flag.
struct GridPlan {
  double* rows[VX_KMAX] = {};
  int64_t rstride[VX_KMAX] = {};
  int64_t cstride[VX_KMAX] = {};
  int32_t* parent[VX_KMAX] = {};
  int64_t* cstart[VX_KMAX] = {};
  int64_t* clen[VX_KMAX] = {};
  unsigned int* bad = nullptr;
};

static void plan_grid(Arena& A, GridPlan& Gp, const vx_csf* grid, int dmax) {
  const int k = grid->k;
  for (int l = 0; l + 1 < k; l++) {  // depth l+1: tuples of dimension k-l-1, l+2 planes
    const int64_t ent = gbinom(dmax + k - l - 1, k - l - 1);
    Gp.cstride[l] = (ent + 31) / 32 * 32;
    Gp.rstride[l] = Gp.cstride[l] * (l + 2);
    Gp.rows[l] = A.take<double>((size_t)grid->n[l] * Gp.rstride[l] + 1);
  }
  for (int l = 1; l < k; l++) Gp.parent[l] = A.take<int32_t>((size_t)grid->n[l] + 1);
  for (int l = 1; l < k; l++) {  // stage l+1: output tuples of dimension k-l-1
    const int64_t nch = gbinom(dmax + k - l - 1, k - l - 1);
    Gp.cstart[l] = A.take<int64_t>(nch + 1);
    Gp.clen[l] = A.take<int64_t>(nch + 1);
  }
  Gp.bad = A.take<unsigned int>(1);
}

size_t grad_workspace_bytes(const vx_poly* P, int np, const vx_csf* grid, int64_t n) {
  Arena A;
  GradPlan G;
  plan_grad(A, G, P, np);
  A.take<double>((size_t)n * np * VX_KMAX + 1);
  A.take<double>((size_t)n * np + 1);
  if (grid) {
    const int k = grid->k;
    int dmax = 0;
    for (int p = 0; p < np; p++) dmax = P[p].degree > dmax ? P[p].degree : dmax;
    // adjoint rows: depth l nodes hold rows of dimension k - l
    for (int l = 0; l < k; l++) A.take<double>((size_t)grid->n[l] * gbinom(dmax + k - l - 1, k - l - 1) + 1);
    A.take<double>(gbinom(dmax + k, k) + 1);
    GridPlan Gp;
    plan_grid(A, Gp, grid, dmax);
  }
  return A.off + 256;
}

static AxisDom axis_dom(const double* dom, int k) {
  AxisDom ad;
  memset(&ad, 0, sizeof ad);
  for (int j = 0; j < k; j++) {
    ad.lo[j] = dom[2 * j];
    ad.hi[j] = dom[2 * j + 1];
  }
  return ad;
}

// Waves to aim for per stage launch (several per SIMD on 256 CUs).
constexpr int64_t GRID_TARGET_WAVES = 8192;

static int launch_grid_stage(int L, bool grad, const double* in, int64_t in_stride, int64_t in_cstride,
                             const int32_t* parent, const int32_t* labels, double dlo, double dhi, int level,
                             const int64_t* cstart, const int64_t* clen, int64_t nch, int64_t nnode, double* out,
                             int64_t out_stride, int64_t out_cstride, double* f, double* jac, int np, int p, int k,
                             hipStream_t st) {
  const int64_t waves = (nnode + 63) / 64;
  int64_t ng = (GRID_TARGET_WAVES + waves - 1) / waves;
  ng = ng < 1 ? 1 : ng > nch ? nch : ng;
  ng = ng > 1024 ? 1024 : ng;
  const dim3 g((unsigned)((nnode + 255) / 256), (unsigned)ng);
#define VX_GS(LL, GG)                                                                                           \
  hipLaunchKernelGGL((k_grid_stage<LL, GG>), g, dim3(256), 0, st, in, in_stride, in_cstride, parent, labels, dlo, \
                     dhi, level, cstart, clen, nch, (int)ng, nnode, out, out_stride, out_cstride, f, jac, np, p, k)
  switch (L * 2 + (grad ? 1 : 0)) {
    case 2: VX_GS(1, false); break;
    case 3: VX_GS(1, true); break;
    case 4: VX_GS(2, false); break;
    case 5: VX_GS(2, true); break;
    case 6: VX_GS(3, false); break;
    case 7: VX_GS(3, true); break;
    case 8: VX_GS(4, false); break;
    default: VX_GS(4, true); break;
  }
#undef VX_GS
  VX_CHECK_LAUNCH("k_grid_stage");
  return VX_OK;
}

// F (and with `jac` its gradient) at the centres of grid's leaves by the
// amortized stages; bit-identical to k_point_eval at those points.
static int grid_forward(const GradPlan& G, GridPlan& Gp, const vx_poly* P, int np, const vx_csf* grid,
                        const double* dom, double* f, double* jac, hipStream_t st) {
  const int k = grid->k;
  const int64_t n = grid->n[k - 1];
  const bool grad = jac != nullptr;
  for (int l = 1; l < k; l++) {
    const int64_t np_ = grid->n[l - 1];
    hipLaunchKernelGGL(k_grid_parents, dim3((unsigned)((np_ + 255) / 256)), dim3(256), 0, st, grid->ptr[l - 1], np_,
                       Gp.parent[l]);
    VX_CHECK_LAUNCH("k_grid_parents");
  }
  int rc;
  for (int p = 0; p < np; p++) {
    const int d = P[p].degree;
    for (int L = 1; L <= k; L++) {
      const bool leaf = L == k;
      double* out = leaf ? nullptr : Gp.rows[L - 1];
      const int64_t ostride = leaf ? 0 : Gp.rstride[L - 1], ocstride = leaf ? 0 : Gp.cstride[L - 1];
      const double dlo = dom[2 * (L - 1)], dhi = dom[2 * (L - 1) + 1];
      if (L == 1) {  // the root row: the padded coefficient stream, its chains from the stream tables
        rc = launch_grid_stage(1, grad, G.stream[p], 0, 0, nullptr, grid->idx[0], dlo, dhi, grid->level,
                               G.start[p], G.plen[p], stream_chains(k, d), grid->n[0], out, ostride, ocstride, f,
                               jac, np, p, k, st);
      } else {
        const int m_out = k - L;
        const int64_t nch = gbinom(d + m_out, m_out);
        hipLaunchKernelGGL(k_grid_chains, dim3((unsigned)((nch + 255) / 256)), dim3(256), 0, st, m_out, d, nch,
                           Gp.cstart[L - 1], Gp.clen[L - 1]);
        VX_CHECK_LAUNCH("k_grid_chains");
        rc = launch_grid_stage(L, grad, Gp.rows[L - 2], Gp.rstride[L - 2], Gp.cstride[L - 2], Gp.parent[L - 1],
                               grid->idx[L - 1], dlo, dhi, grid->level, Gp.cstart[L - 1], Gp.clen[L - 1], nch,
                               grid->n[L - 1], out, ostride, ocstride, f, jac, np, p, k, st);
      }
      if (rc) return rc;
    }
  }
  (void)n;
  return VX_OK;
}

// VX_OK when x holds, bit for bit, the centres of grid's leaves (waits for
// the stream once).
static int check_centres(GridPlan& Gp, const vx_csf* grid, const double* dom, const double* x, hipStream_t st) {
  const int k = grid->k;
  const int64_t n = grid->n[k - 1];
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, Gp.bad);
  VX_CHECK_LAUNCH("k_zero_u32");
  hipLaunchKernelGGL(k_check_centres, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, k, grid->level,
                     grid->idx[0], grid->idx[1], grid->idx[2], grid->idx[3], grid->ptr[0], grid->ptr[1], grid->ptr[2],
                     grid->n[0], grid->n[1], grid->n[2], n, axis_dom(dom, k), x, Gp.bad);
  VX_CHECK_LAUNCH("k_check_centres");
  unsigned int bad = 0;
  VX_HIP(hipMemcpyAsync(&bad, Gp.bad, sizeof bad, hipMemcpyDeviceToHost, st));
  VX_HIP(hipStreamSynchronize(st));
  if (bad) VX_FAIL(VX_EINVAL, "the points are not the centres of the grid's leaves");
  return VX_OK;
}

static StreamSet stream_set(const GradPlan& G, const vx_poly* P, int np) {
  StreamSet ss;
  memset(&ss, 0, sizeof ss);
  for (int p = 0; p < np; p++) {
    ss.s[p] = G.stream[p];
    ss.d[p] = P[p].degree;
  }
  return ss;
}

// xbar[i][j] = sum_p gbar[p][i] jac[i][p][j]
__global__ void k_contract_xbar(int np, int k, int64_t n, const double* __restrict__ gbar,
                                const double* __restrict__ jac, double* __restrict__ xbar) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int j = 0; j < k; j++) {
    double s = 0.0;
    for (int p = 0; p < np; p++) s += gbar[p * n + i] * jac[(i * np + p) * k + j];
    xbar[i * k + j] = s;
  }
}

int grad_impl(const vx_poly* P, int np, const double* x, int64_t n, double* f, double* jac, const double* gbar,
              double* xbar, double* dcoef, const vx_csf* grid, const double* dom, void* ws, size_t ws_bytes,
              hipStream_t st) {
  const int k = P[0].k;
  Arena A;
  A.base = reinterpret_cast<char*>(ws);
  A.size = ws_bytes;
  GradPlan G;
  plan_grad(A, G, P, np);
  double* rows[VX_KMAX] = {};
  double* root = nullptr;
  int dmax = 0;
  for (int p = 0; p < np; p++) dmax = P[p].degree > dmax ? P[p].degree : dmax;
  if (grid) {
    for (int l = 0; l < k; l++) rows[l] = A.take<double>((size_t)grid->n[l] * gbinom(dmax + k - l - 1, k - l - 1) + 1);
    root = A.take<double>(gbinom(dmax + k, k) + 1);
  }
  double* jac_tmp = nullptr;
  if (xbar && !jac) jac_tmp = A.take<double>((size_t)n * np * k + 1);
  GridPlan Gp;
  if (grid) plan_grid(A, Gp, grid, dmax);
  double* f_tmp = (n > 0 && !f) ? A.take<double>((size_t)n * np + 1) : nullptr;
  if (A.overflow) VX_FAIL(VX_ECAPACITY, "eval_grad: workspace of %zu bytes is too small (%zu needed)", ws_bytes, A.off + 256);
  int rc;
  if (grid && x && n > 0 && (rc = check_centres(Gp, grid, dom, x, st))) return rc;
  if ((rc = build_streams(G, P, np, st))) return rc;
  const StreamSet ss = stream_set(G, P, np);
  if (jac_tmp) jac = jac_tmp;
  if (n > 0 && (f || jac) && grid) {
    if (!f) f = f_tmp;
    if ((rc = grid_forward(G, Gp, P, np, grid, dom, f, jac, st))) return rc;
  } else if (n > 0 && (f || jac)) {
    if (!f) f = f_tmp;
    dim3 grid3((unsigned)((n + 64 * PPL - 1) / (64 * PPL)), (unsigned)np);
    const bool gradf = jac != nullptr;
#define VX_PE(KK)                                                                                       \
  if (gradf)                                                                                            \
    hipLaunchKernelGGL((k_point_eval<KK, true>), grid3, dim3(64), 0, st, ss, np, x, n, f, jac);         \
  else                                                                                                  \
    hipLaunchKernelGGL((k_point_eval<KK, false>), grid3, dim3(64), 0, st, ss, np, x, n, f, jac);
    switch (k) {
      case 1: VX_PE(1) break;
      case 2: VX_PE(2) break;
      case 3: VX_PE(3) break;
      default: VX_PE(4) break;
    }
#undef VX_PE
    VX_CHECK_LAUNCH("k_point_eval");
  }
  if (xbar && n > 0) {
    hipLaunchKernelGGL(k_contract_xbar, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, np, k, n, gbar,
                       (const double*)jac, xbar);
    VX_CHECK_LAUNCH("k_contract_xbar");
  }
  if (dcoef && gbar) {
    if (!grid) VX_FAIL(VX_EUNSUPPORTED, "eval_grad: coefficient gradients need points given as a CSF grid");
    for (int p = 0; p < np; p++) {
      const int d = P[p].degree;
      // leaves -> depth k-1 rows (dimension 1) -> ... -> root row (dimension k)
      const double* in = gbar + (int64_t)p * grid->n[k - 1];
      int64_t in_stride = 1;
      for (int l = k - 1; l >= 0; l--) {
        const int m_in = k - 1 - l;
        const int64_t nout = gbinom(d + m_in + 1, m_in + 1);
        const int64_t nparent = l == 0 ? 1 : grid->n[l - 1];
        double* out = l == 0 ? root : rows[l - 1];
        // input rows staged in LDS where they are short: 1 entry (gbar) at the
        // leaf depth, d + 1 one depth up
        int stage_w = m_in == 0 ? 1 : (m_in == 1 ? (int)in_stride : 0);
        if (adjoint_lds_bytes(d, stage_w) > ADJ_LDS_MAX) stage_w = 0;
        const int threads = nout <= 128 ? 128 : 256;
        dim3 g2((unsigned)nparent, (unsigned)((nout + threads - 1) / threads));
        hipLaunchKernelGGL(k_adjoint_level, g2, dim3(threads), adjoint_lds_bytes(d, stage_w), st, d, m_in,
                           l == 0 ? nullptr : grid->ptr[l - 1], grid->n[0], grid->idx[l], dom[2 * l], dom[2 * l + 1],
                           grid->level, in, in_stride, out, nout, nout, stage_w);
        VX_CHECK_LAUNCH("k_adjoint_level");
        in = out;
        in_stride = nout;
      }
      int64_t cube = 1;
      for (int i = 0; i < k; i++) cube *= P[p].side;
      double* dc = dcoef + (int64_t)p * cube;
      VX_HIP(hipMemsetAsync(dc, 0, sizeof(double) * cube, st));
      const int64_t nrow = gbinom(d + k, k);
      hipLaunchKernelGGL(k_adjoint_scatter, dim3((unsigned)((nrow + 255) / 256)), dim3(256), 0, st, k, d, P[p].side,
                         (const double*)root, nrow, dc);
      VX_CHECK_LAUNCH("k_adjoint_scatter");
    }
  }
  return VX_OK;
}

int newton_impl(const vx_poly* P, int np, double* x, int64_t n, int steps, double* f, void* ws, size_t ws_bytes,
                hipStream_t st, const vx_csf* grid, const double* dom) {
  const int k = P[0].k;
  Arena A;
  A.base = reinterpret_cast<char*>(ws);
  A.size = ws_bytes;
  GradPlan G;
  plan_grad(A, G, P, np);
  // the same layout as grad_workspace_bytes(P, np, grid, n)
  double* j0 = A.take<double>((size_t)n * np * VX_KMAX + 1);
  double* f0 = A.take<double>((size_t)n * np + 1);
  GridPlan Gp;
  if (grid) {
    int dmax = 0;
    for (int p = 0; p < np; p++) dmax = P[p].degree > dmax ? P[p].degree : dmax;
    for (int l = 0; l < k; l++) A.take<double>((size_t)grid->n[l] * gbinom(dmax + k - l - 1, k - l - 1) + 1);
    A.take<double>(gbinom(dmax + k, k) + 1);
    plan_grid(A, Gp, grid, dmax);
  }
  if (A.overflow) VX_FAIL(VX_ECAPACITY, "newton_project: workspace too small (%zu needed)", A.off + 256);
  int rc;
  if (grid && n > 0 && (rc = check_centres(Gp, grid, dom, x, st))) return rc;
  if ((rc = build_streams(G, P, np, st))) return rc;
  const StreamSet ss = stream_set(G, P, np);
  if (n == 0) return VX_OK;
  if (grid && (rc = grid_forward(G, Gp, P, np, grid, dom, f0, j0, st))) return rc;
  const double* F0 = grid ? f0 : nullptr;
  const double* J0 = grid ? j0 : nullptr;
  dim3 g1((unsigned)((n + 64 * PPL - 1) / (64 * PPL)));
  if (steps > 0) {
    switch (k) {
      case 1: hipLaunchKernelGGL(k_newton<1>, g1, dim3(64), 0, st, ss, np, x, n, steps, F0, J0); break;
      case 2: hipLaunchKernelGGL(k_newton<2>, g1, dim3(64), 0, st, ss, np, x, n, steps, F0, J0); break;
      case 3: hipLaunchKernelGGL(k_newton<3>, g1, dim3(64), 0, st, ss, np, x, n, steps, F0, J0); break;
      default: hipLaunchKernelGGL(k_newton<4>, g1, dim3(64), 0, st, ss, np, x, n, steps, F0, J0); break;
    }
    VX_CHECK_LAUNCH("k_newton");
  }
  if (!f) return VX_OK;
  if (steps == 0 && F0) {  // the points have not moved: F is the grid's
    VX_HIP(hipMemcpyAsync(f, F0, sizeof(double) * (size_t)n * np, hipMemcpyDeviceToDevice, st));
    return VX_OK;
  }
  // values at the final points, without the derivative chains
  const dim3 g2((unsigned)((n + 64 * PPL - 1) / (64 * PPL)), (unsigned)np);
  switch (k) {
    case 1: hipLaunchKernelGGL((k_point_eval<1, false>), g2, dim3(64), 0, st, ss, np, x, n, f, nullptr); break;
    case 2: hipLaunchKernelGGL((k_point_eval<2, false>), g2, dim3(64), 0, st, ss, np, x, n, f, nullptr); break;
    case 3: hipLaunchKernelGGL((k_point_eval<3, false>), g2, dim3(64), 0, st, ss, np, x, n, f, nullptr); break;
    default: hipLaunchKernelGGL((k_point_eval<4, false>), g2, dim3(64), 0, st, ss, np, x, n, f, nullptr); break;
  }
  VX_CHECK_LAUNCH("k_point_eval");
  return VX_OK;
}

int centres_impl(const vx_csf* S, const double* dom, double* x, hipStream_t st) {
  const int k = S->k;
  const int64_t n = S->n[k - 1];
  if (n == 0) return VX_OK;
  const AxisDom ad = axis_dom(dom, k);
  hipLaunchKernelGGL(k_csf_centres, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, k, S->level, S->idx[0],
                     S->idx[1], S->idx[2], S->idx[3], S->ptr[0], S->ptr[1], S->ptr[2], S->n[0], S->n[1], S->n[2], n,
                     ad, x);
  VX_CHECK_LAUNCH("k_csf_centres");
  return VX_OK;
}

}  // namespace vx
