// The criteria of Sec. 3.2 beyond C0: Taylor-form exclusion tests (orders 1
// and 2), the inclusion criterion C1 (vertex signs and its Taylor form) and
// the Newton interval test for square systems.
//
// Mean-value exclusion test: the Taylor form of order 1 (Sec. 3.2 of Moroz,
// arXiv 2406.09857, Taylor form definition with m = 1),
//   T(F, B) = F(c) + sum_i dF/dx_i(B) * (B_i - c_i),   c the centre of B,
// evaluated with outward rounding.  Every part reuses the amortized CSF
// evaluation (Algorithm 2) on the level's box CSF:
//   - F(c): the same polynomial evaluated on the degenerate boxes of the cell
//     centres (exact dyadics on [-1,1]^k);
//   - dF/dx_i(B): the derivative polynomials, whose coefficients
//     (e_i + 1) c_{e + u_i} are rounded outward into interval coefficients,
//     evaluated on the boxes;
//   - B_i - c_i = [RD(lo_i - chi_i), RU(hi_i - clo_i)] from the cell and
//     centre enclosures, and the sum taken left to right over i.
// A box is dropped when, for some polynomial, 0 lies outside T(F, B); the
// test is combined with C0 by AND-ing keep flags.
//
// Order 2 (the same definition with m = 2):
//   T2(F, B) = F(c) + sum_i dF/dx_i(c) W_i + sum_{i<=j} H_ij(B) X_ij,
// W_i = B_i - c_i, H_ii = (1/2) d2F/dx_i^2, H_ij = d2F/dx_i dx_j (i < j),
// X_ii = W_i^2 (the range of a square, [0, max(a^2, b^2)] when W_i holds 0),
// X_ij = W_i W_j; the gradient is evaluated at the centre enclosures and the
// H_ij on the boxes, all by Algorithm 2 on the level's CSF, and the terms are
// added left to right, the pairs in lexicographic order.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "common.hpp"
#include "eval.hpp"
#include "interval.hpp"
#include "profile.hpp"
#include "scan.hpp"

namespace vx {

// Derivative coefficient cubes, one thread per (derivative, entry).  Entry e
// of dF_p/dx_i is [RD(n * clo), RU(n * chi)] of source entry e + u_i with
// n = e_i + 1 (> 0, so the bounds scale separately); zero outside the
// simplex of degree d - 1.  Output cubes keep the input side.
struct DerivArgs {
  const double* clo[VX_MAXPOLY];
  const double* chi[VX_MAXPOLY];
  int d[VX_MAXPOLY];
  int side[VX_MAXPOLY];
};

__global__ void k_deriv(DerivArgs a, int k, int64_t cube_max, double* __restrict__ olo, double* __restrict__ ohi) {
  round_up_mode();
  const int p = blockIdx.y / k, axis = blockIdx.y % k;
  const int side = a.side[p], d = a.d[p];
  int64_t total = 1;
  for (int j = 0; j < k; j++) total *= side;
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= total) return;
  int64_t q = f, stride = 1, astride = 0;
  int deg = 0, ea = 0;
  for (int j = k - 1; j >= 0; j--) {
    const int e = (int)(q % side);
    q /= side;
    deg += e;
    if (j == axis) {
      ea = e;
      astride = stride;
    }
    stride *= side;
  }
  double* lo = olo + (int64_t)blockIdx.y * cube_max;
  double* hi = ohi + (int64_t)blockIdx.y * cube_max;
  if (deg + 1 > d || ea + 1 >= side) {
    lo[f] = 0.0;
    hi[f] = 0.0;
    return;
  }
  const double n = (double)(ea + 1);
  const int64_t src = f + astride;
  const double cl = a.clo[p][src];
  const double ch = a.chi[p] ? a.chi[p][src] : cl;
  lo[f] = -opaque(n * opaque(-cl));  // RD(n * cl) = -RU(n * -cl)
  hi[f] = n * ch;
}

// Second-derivative coefficient cubes, one thread per (polynomial, pair,
// entry); the pairs (i, j), i <= j, in lexicographic order.  Entry e of H_ij
// is [RD(m clo), RU(m chi)] of source entry e + u_i + u_j with the integer
// m = (e_i+1)(e_i+2)/2 (i == j) or (e_i+1)(e_j+1), exact in double; zero
// outside the simplex of degree d - 2.
struct PairTab {
  int8_t i[VX_KMAX * (VX_KMAX + 1) / 2];
  int8_t j[VX_KMAX * (VX_KMAX + 1) / 2];
  int n;
};

__global__ void k_deriv2(DerivArgs a, int k, PairTab pt, int64_t cube_max, double* __restrict__ olo,
                         double* __restrict__ ohi) {
  round_up_mode();
  const int p = blockIdx.y / pt.n, t = blockIdx.y % pt.n;
  const int ai = pt.i[t], aj = pt.j[t];
  const int side = a.side[p], d = a.d[p];
  int64_t total = 1;
  for (int j = 0; j < k; j++) total *= side;
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= total) return;
  int64_t q = f, stride = 1, shift = 0;
  int deg = 0, ei = 0, ej = 0;
  for (int j = k - 1; j >= 0; j--) {
    const int e = (int)(q % side);
    q /= side;
    deg += e;
    if (j == ai) {
      ei = e;
      shift += stride;
    }
    if (j == aj) {
      ej = e;
      shift += stride;
    }
    stride *= side;
  }
  double* lo = olo + (int64_t)blockIdx.y * cube_max;
  double* hi = ohi + (int64_t)blockIdx.y * cube_max;
  if (deg + 2 > d || ei + (ai == aj ? 2 : 1) >= side || ej + 1 >= side) {
    lo[f] = 0.0;
    hi[f] = 0.0;
    return;
  }
  const double m = ai == aj ? (double)((ei + 1) * (ei + 2) / 2) : (double)((ei + 1) * (ej + 1));
  const int64_t src = f + shift;
  const double cl = a.clo[p][src];
  const double ch = a.chi[p] ? a.chi[p][src] : cl;
  lo[f] = -opaque(m * opaque(-cl));  // RD(m * cl) = -RU(m * -cl)
  hi[f] = m * ch;
}

// Labels of every leaf on every axis: walk up the CSF by binary search.
struct CsfView {
  const int32_t* idx[VX_KMAX];
  const int32_t* ptr[VX_KMAX];
  int64_t n[VX_KMAX];
};

__global__ void k_leaf_labels(int k, CsfView c, int32_t* __restrict__ labels) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nleaf = c.n[k - 1];
  if (b >= nleaf) return;
  const int32_t* const* idx = c.idx;
  const int32_t* const* ptr = c.ptr;
  const int64_t* n = c.n;
  int64_t q = b;
  for (int l = k - 1; l >= 0; l--) {
    labels[b * k + l] = idx[l][q];
    if (l > 0) {
      int64_t lo = 0, hi = n[l - 1];  // last parent with ptr[l-1][parent] <= q
      while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (ptr[l - 1][mid] <= q) lo = mid; else hi = mid;
      }
      q = lo;
    }
  }
}

struct GridSet {
  AxisGrid cell[VX_KMAX];
  AxisGrid centre[VX_KMAX];
  AxisGrid vertex[VX_KMAX];
};

// T(F_p, B) for every leaf and polynomial; keep (if given) is AND-ed with
// "0 in T(F_p, B) for every p" (NaN endpoints never exclude).
__global__ void k_mv_combine(int k, int np, int64_t nleaf, GridSet gs, const int32_t* __restrict__ labels,
                             const double* __restrict__ fc_lo, const double* __restrict__ fc_hi,
                             const double* __restrict__ d_lo, const double* __restrict__ d_hi,
                             double* __restrict__ lo, double* __restrict__ hi, uint8_t* __restrict__ keep) {
  round_up_mode();
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nleaf) return;
  CellOps W[VX_KMAX];
  for (int i = 0; i < k; i++) {
    double inl, ih, cnl, ch;
    const int32_t lab = labels[b * k + i];
    cell(gs.cell[i], lab, inl, ih);
    cell(gs.centre[i], lab, cnl, ch);
    const double wnl = ch + inl;  // -RD(lo_i - chi_i) = RU(chi_i - lo_i)
    const double wh = ih + cnl;   // RU(hi_i - clo_i)
    W[i] = cell_ops(wnl, wh, CLS_STRADDLE);
  }
  bool excl = false;
  for (int p = 0; p < np; p++) {
    double anl = -opaque(fc_lo[(int64_t)p * nleaf + b]);
    double ah = fc_hi[(int64_t)p * nleaf + b];
    for (int i = 0; i < k; i++) {
      const int64_t di = ((int64_t)p * k + i) * nleaf + b;
      double dnl = -opaque(d_lo[di]);
      double dh = d_hi[di];
      mul_add_sep(dnl, dh, W[i], anl, ah);  // D_i * W_i + acc
      anl = dnl;
      ah = dh;
    }
    const double l = -opaque(anl);
    lo[(int64_t)p * nleaf + b] = l;
    hi[(int64_t)p * nleaf + b] = ah;
    excl = excl || (l > 0.0) || (ah < 0.0);
  }
  if (keep && excl) keep[b] = 0;
}

// Range of x^2 over X = [lo, hi] held as (nlo, hi): [RD(lo^2), RU(hi^2)] when
// lo >= 0, [RD(hi^2), RU(lo^2)] when hi <= 0, else [0, RU(max(lo^2, hi^2))].
__device__ __forceinline__ void interval_square(double xnl, double xh, double& snl, double& sh) {
  if (xnl <= 0.0) {         // lo >= 0
    snl = xnl * opaque(-xnl);  // RU(-lo^2)
    sh = xh * xh;
  } else if (xh <= 0.0) {
    snl = xh * opaque(-xh);    // RU(-hi^2)
    sh = xnl * xnl;            // RU(lo^2)
  } else {
    snl = 0.0;
    sh = fmax(xnl * xnl, xh * xh);
  }
}

// T2(F_p, B) for every leaf and polynomial; keep (if given) is AND-ed with
// "0 in T2(F_p, B) for every p" (NaN endpoints never exclude).  Layouts:
// fc (np x nleaf), dc ((p, i) x nleaf), h ((p, pair) x nleaf).
__global__ void k_t2_combine(int k, int np, int64_t nleaf, GridSet gs, const int32_t* __restrict__ labels,
                             const double* __restrict__ fc_lo, const double* __restrict__ fc_hi,
                             const double* __restrict__ dc_lo, const double* __restrict__ dc_hi,
                             const double* __restrict__ h_lo, const double* __restrict__ h_hi,
                             double* __restrict__ lo, double* __restrict__ hi, uint8_t* __restrict__ keep) {
  round_up_mode();
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nleaf) return;
  double wnl[VX_KMAX], wh[VX_KMAX];
  CellOps W[VX_KMAX];
  for (int i = 0; i < k; i++) {
    double inl, ih, cnl, ch;
    const int32_t lab = labels[b * k + i];
    cell(gs.cell[i], lab, inl, ih);
    cell(gs.centre[i], lab, cnl, ch);
    wnl[i] = ch + inl;  // -RD(lo_i - chi_i) = RU(chi_i - lo_i)
    wh[i] = ih + cnl;   // RU(hi_i - clo_i)
    W[i] = cell_ops(wnl[i], wh[i], CLS_STRADDLE);
  }
  const int npair = k * (k + 1) / 2;
  bool excl = false;
  for (int p = 0; p < np; p++) {
    double anl = -opaque(fc_lo[(int64_t)p * nleaf + b]);
    double ah = fc_hi[(int64_t)p * nleaf + b];
    for (int i = 0; i < k; i++) {
      const int64_t di = ((int64_t)p * k + i) * nleaf + b;
      double dnl = -opaque(dc_lo[di]);
      double dh = dc_hi[di];
      mul_add_sep(dnl, dh, W[i], anl, ah);  // Dc_i * W_i + acc
      anl = dnl;
      ah = dh;
    }
    int t = 0;
    for (int i = 0; i < k; i++)
      for (int j = i; j < k; j++, t++) {
        double xnl, xh;
        if (i == j) {
          interval_square(wnl[i], wh[i], xnl, xh);
        } else {
          xnl = wnl[i];
          xh = wh[i];
          mul_add_sep(xnl, xh, W[j], 0.0, 0.0);  // W_i * W_j (+ 0: exact)
        }
        const CellOps X = cell_ops(xnl, xh, CLS_STRADDLE);
        const int64_t hi_ = ((int64_t)p * npair + t) * nleaf + b;
        double hnl = -opaque(h_lo[hi_]);
        double hh = h_hi[hi_];
        mul_add_sep(hnl, hh, X, anl, ah);  // H_t * X_t + acc
        anl = hnl;
        ah = hh;
      }
    const double l = -opaque(anl);
    lo[(int64_t)p * nleaf + b] = l;
    hi[(int64_t)p * nleaf + b] = ah;
    excl = excl || (l > 0.0) || (ah < 0.0);
  }
  if (keep && excl) keep[b] = 0;
}

// Order-2 bound of F at a point V of the box: F(c) + sum_i Dc_i W_i +
// sum_t H_t X_t with W_i = V_i - c_i (both held as (nlo, hi)), the same sum
// as k_t2_combine.
__device__ __forceinline__ void t2_at(int k, int np_, int p, int64_t nleaf, int64_t b, double fnl, double fh,
                                      const double* __restrict__ dc_lo, const double* __restrict__ dc_hi,
                                      const double* __restrict__ h_lo, const double* __restrict__ h_hi,
                                      const double* wnl, const double* wh, double& rnl, double& rh) {
  (void)np_;
  const int npair = k * (k + 1) / 2;
  double anl = fnl, ah = fh;
  for (int i = 0; i < k; i++) {
    const int64_t di = ((int64_t)p * k + i) * nleaf + b;
    double dnl = -opaque(dc_lo[di]);
    double dh = dc_hi[di];
    mul_add_sep(dnl, dh, cell_ops(wnl[i], wh[i], CLS_STRADDLE), anl, ah);
    anl = dnl;
    ah = dh;
  }
  int t = 0;
  for (int i = 0; i < k; i++)
    for (int j = i; j < k; j++, t++) {
      double xnl, xh;
      if (i == j) {
        interval_square(wnl[i], wh[i], xnl, xh);
      } else {
        xnl = wnl[i];
        xh = wh[i];
        mul_add_sep(xnl, xh, cell_ops(wnl[j], wh[j], CLS_STRADDLE), 0.0, 0.0);
      }
      const int64_t hi_ = ((int64_t)p * npair + t) * nleaf + b;
      double hnl = -opaque(h_lo[hi_]);
      double hh = h_hi[hi_];
      mul_add_sep(hnl, hh, cell_ops(xnl, xh, CLS_STRADDLE), anl, ah);
      anl = hnl;
      ah = hh;
    }
  rnl = anl;
  rh = ah;
}

// Taylor-based inclusion criterion (order 2): incl[p * nleaf + b] = 1 when
// the order-2 bound of F_p at the vertex maximizing the linear part
// F(c) + grad F(c).(x - c) is > 0 and at the vertex minimizing it is < 0.
// On axis i the maximizing vertex takes the upper end when the enclosure of
// dF/dx_i(c) has lo + hi >= 0 (nlo <= hi, exactly), else the lower end.
__global__ void k_t2_inclusion(int k, int np, int64_t nleaf, GridSet gs, const int32_t* __restrict__ labels,
                               const double* __restrict__ fc_lo, const double* __restrict__ fc_hi,
                               const double* __restrict__ dc_lo, const double* __restrict__ dc_hi,
                               const double* __restrict__ h_lo, const double* __restrict__ h_hi,
                               uint8_t* __restrict__ incl) {
  round_up_mode();
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nleaf) return;
  // per axis: the lower and upper vertex as V - c
  double lnl[VX_KMAX], lh[VX_KMAX], unl[VX_KMAX], uh[VX_KMAX];
  for (int i = 0; i < k; i++) {
    double cnl, ch, vnl, vh;
    const int32_t lab = labels[b * k + i];
    cell(gs.centre[i], lab, cnl, ch);
    cell(gs.vertex[i], lab, vnl, vh);
    lnl[i] = ch + vnl;  // -RD(v_lo - chi)
    lh[i] = vh + cnl;   // RU(v_hi - clo)
    cell(gs.vertex[i], lab + 1, vnl, vh);
    unl[i] = ch + vnl;
    uh[i] = vh + cnl;
  }
  for (int p = 0; p < np; p++) {
    double xnl[VX_KMAX], xh[VX_KMAX], nnl[VX_KMAX], nh[VX_KMAX];  // V_max - c, V_min - c
    for (int i = 0; i < k; i++) {
      const int64_t di = ((int64_t)p * k + i) * nleaf + b;
      const bool up = -dc_lo[di] <= dc_hi[di];
      xnl[i] = up ? unl[i] : lnl[i];
      xh[i] = up ? uh[i] : lh[i];
      nnl[i] = up ? lnl[i] : unl[i];
      nh[i] = up ? lh[i] : uh[i];
    }
    const double fnl = -opaque(fc_lo[(int64_t)p * nleaf + b]);
    const double fh = fc_hi[(int64_t)p * nleaf + b];
    double mxnl, mxh, mnnl, mnh;
    t2_at(k, np, p, nleaf, b, fnl, fh, dc_lo, dc_hi, h_lo, h_hi, xnl, xh, mxnl, mxh);
    t2_at(k, np, p, nleaf, b, fnl, fh, dc_lo, dc_hi, h_lo, h_hi, nnl, nh, mnnl, mnh);
    // lower bound at V_max > 0 (nlo < 0) and upper bound at V_min < 0
    incl[(int64_t)p * nleaf + b] = (uint8_t)((-opaque(mxnl) > 0.0) && (mnh < 0.0));
  }
}

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------
struct MvPolys {
  int order = 1;
  std::vector<vx_poly> dp;  // first-derivative polynomials, (p, axis) order
  std::vector<vx_poly> hp;  // order 2: H_ij polynomials, (p, pair) order
  int64_t cube_max = 1;
};

static int npairs(int k) { return k * (k + 1) / 2; }

// Coefficient cube pointers are null when only sizes are wanted.
static MvPolys mv_polys(const vx_poly* P, int np, int order, double* dlo, double* dhi, double* hlo, double* hhi) {
  MvPolys M;
  M.order = order;
  const int k = P[0].k;
  for (int p = 0; p < np; p++) {
    int64_t cube = 1;
    for (int j = 0; j < k; j++) cube *= P[p].side;
    M.cube_max = cube > M.cube_max ? cube : M.cube_max;
  }
  for (int p = 0; p < np; p++)
    for (int i = 0; i < k; i++) {
      vx_poly q;
      memset(&q, 0, sizeof q);
      q.k = k;
      q.degree = P[p].degree > 0 ? P[p].degree - 1 : 0;
      q.side = P[p].side;
      const int64_t slot = (int64_t)p * k + i;
      q.c_lo = dlo ? dlo + slot * M.cube_max : nullptr;
      q.c_hi = dhi ? dhi + slot * M.cube_max : nullptr;
      M.dp.push_back(q);
    }
  if (order == 2)
    for (int p = 0; p < np; p++)
      for (int t = 0; t < npairs(k); t++) {
        vx_poly q;
        memset(&q, 0, sizeof q);
        q.k = k;
        q.degree = P[p].degree > 1 ? P[p].degree - 2 : 0;
        q.side = P[p].side;
        const int64_t slot = (int64_t)p * npairs(k) + t;
        q.c_lo = hlo ? hlo + slot * M.cube_max : nullptr;
        q.c_hi = hhi ? hhi + slot * M.cube_max : nullptr;
        M.hp.push_back(q);
      }
  return M;
}

static DerivArgs deriv_args(const vx_poly* P, int np) {
  DerivArgs a;
  memset(&a, 0, sizeof a);
  for (int p = 0; p < np; p++) {
    a.clo[p] = P[p].c_lo;
    a.chi[p] = P[p].c_hi;
    a.d[p] = P[p].degree;
    a.side[p] = P[p].side;
  }
  return a;
}

static int launch_deriv(const vx_poly* P, int np, const MvPolys& M, double* dlo, double* dhi, hipStream_t st) {
  const int k = P[0].k;
  hipLaunchKernelGGL(k_deriv, dim3((unsigned)((M.cube_max + 255) / 256), (unsigned)(np * k)), dim3(256), 0, st,
                     deriv_args(P, np), k, M.cube_max, dlo, dhi);
  VX_CHECK_LAUNCH("k_deriv");
  return VX_OK;
}

static int launch_deriv2(const vx_poly* P, int np, const MvPolys& M, double* hlo, double* hhi, hipStream_t st) {
  const int k = P[0].k;
  PairTab pt;
  memset(&pt, 0, sizeof pt);
  for (int i = 0; i < k; i++)
    for (int j = i; j < k; j++, pt.n++) {
      pt.i[pt.n] = (int8_t)i;
      pt.j[pt.n] = (int8_t)j;
    }
  hipLaunchKernelGGL(k_deriv2, dim3((unsigned)((M.cube_max + 255) / 256), (unsigned)(np * pt.n)), dim3(256), 0,
                     st, deriv_args(P, np), k, pt, M.cube_max, hlo, hhi);
  VX_CHECK_LAUNCH("k_deriv2");
  return VX_OK;
}

// Per-run state of a Taylor test: derivative coefficient cubes and the
// prepared tables of F and of its derivatives (built once).
struct MvRun {
  MvPolys M;
  Prepared QF, QD, QH;
  double* dlo = nullptr;
  double* dhi = nullptr;
  double* hlo = nullptr;
  double* hhi = nullptr;
};

static size_t cubes_bytes(const MvPolys& M, int64_t count) {
  return (sizeof(double) * (size_t)M.cube_max * count + 255) / 256 * 256;
}

static size_t mv_run_bytes(const vx_poly* P, int np, int order) {
  MvPolys M = mv_polys(P, np, order, nullptr, nullptr, nullptr, nullptr);
  const int k = P[0].k;
  size_t b = cubes_bytes(M, (int64_t)np * k) * 2 + prepared_bytes(P, np) + prepared_bytes(M.dp.data(), (int)M.dp.size());
  if (order == 2) b += cubes_bytes(M, (int64_t)np * npairs(k)) * 2 + prepared_bytes(M.hp.data(), (int)M.hp.size());
  return b + 2048;
}

static int mv_run_prepare(const vx_poly* P, int np, int order, char* ws, size_t bytes, MvRun& R, hipStream_t st) {
  const int k = P[0].k;
  MvPolys M0 = mv_polys(P, np, order, nullptr, nullptr, nullptr, nullptr);
  const size_t cd = cubes_bytes(M0, (int64_t)np * k);
  const size_t ch = order == 2 ? cubes_bytes(M0, (int64_t)np * npairs(k)) : 0;
  R.dlo = reinterpret_cast<double*>(ws);
  R.dhi = reinterpret_cast<double*>(ws + cd);
  R.hlo = order == 2 ? reinterpret_cast<double*>(ws + 2 * cd) : nullptr;
  R.hhi = order == 2 ? reinterpret_cast<double*>(ws + 2 * cd + ch) : nullptr;
  R.M = mv_polys(P, np, order, R.dlo, R.dhi, R.hlo, R.hhi);
  char* at = ws + 2 * cd + 2 * ch;
  const size_t qf = (prepared_bytes(P, np) + 255) / 256 * 256;
  const size_t qd = (prepared_bytes(R.M.dp.data(), (int)R.M.dp.size()) + 255) / 256 * 256;
  const size_t qh = order == 2 ? (prepared_bytes(R.M.hp.data(), (int)R.M.hp.size()) + 255) / 256 * 256 : 0;
  if (2 * cd + 2 * ch + qf + qd + qh > bytes) VX_FAIL(VX_ECAPACITY, "Taylor test: workspace too small");
  int rc;
  if ((rc = launch_deriv(P, np, R.M, R.dlo, R.dhi, st))) return rc;
  if (order == 2 && (rc = launch_deriv2(P, np, R.M, R.hlo, R.hhi, st))) return rc;
  if ((rc = prepare_polys(P, np, at, qf, &R.QF, st))) return rc;
  if ((rc = prepare_polys(R.M.dp.data(), (int)R.M.dp.size(), at + qf, qd, &R.QD, st))) return rc;
  if (order == 2 && (rc = prepare_polys(R.M.hp.data(), (int)R.M.hp.size(), at + qf + qd, qh, &R.QH, st))) return rc;
  return VX_OK;
}

static size_t mv_scratch_bytes(const vx_poly* P, int np, const MvPolys& M, const vx_csf* S) {
  size_t e = eval_level_bytes(P, np, S);
  const size_t ed = eval_level_bytes(M.dp.data(), (int)M.dp.size(), S);
  e = ed > e ? ed : e;
  if (M.order == 2) {
    const size_t eh = eval_level_bytes(M.hp.data(), (int)M.hp.size(), S);
    e = eh > e ? eh : e;
  }
  return e;
}

static size_t mv_level_bytes(const vx_poly* P, int np, const MvPolys& M, const vx_csf* S) {
  const int k = S->k;
  const int64_t nl = S->n[k - 1];
  auto r = [](size_t b) { return (b + 255) / 256 * 256; };
  size_t b = r(sizeof(double) * np * nl) * 2 + r(sizeof(double) * np * k * nl) * 2 + r(sizeof(int32_t) * k * nl) +
             mv_scratch_bytes(P, np, M, S) + 256;
  if (M.order == 2) b += r(sizeof(double) * np * npairs(k) * nl) * 2;
  return b;
}

// One level: Taylor enclosures lo/hi (np x nleaf) and keep AND-ed.
// With `incl` (order 2 only) the Taylor-based inclusion flags are written
// instead of the enclosures.
static int mv_level(const vx_poly* P, int np, const MvRun& R, const vx_csf* S, const double* dom, double* lo,
                    double* hi, uint8_t* keep, char* ws, size_t bytes, hipStream_t st, uint8_t* incl = nullptr) {
  const int k = S->k;
  const int64_t nl = S->n[k - 1];
  if (nl == 0) return VX_OK;
  const bool t2 = R.M.order == 2;
  Arena A;
  A.base = ws;
  A.size = bytes;
  double* fcl = A.take<double>((size_t)np * nl);
  double* fch = A.take<double>((size_t)np * nl);
  double* dl = A.take<double>((size_t)np * k * nl);
  double* dh = A.take<double>((size_t)np * k * nl);
  double* hl = t2 ? A.take<double>((size_t)np * npairs(k) * nl) : nullptr;
  double* hh = t2 ? A.take<double>((size_t)np * npairs(k) * nl) : nullptr;
  int32_t* labels = A.take<int32_t>((size_t)k * nl);
  const size_t sb = mv_scratch_bytes(P, np, R.M, S);
  char* scratch = A.take<char>(sb);
  if (A.overflow) VX_FAIL(VX_ECAPACITY, "Taylor test: workspace of %zu bytes is too small", bytes);
  const int pr = prof_start(t2 ? "taylor2" : "mean_value", (double)nl, st);
  int rc;
  // F at the centres; the gradient on the boxes (order 1) or at the centres
  // (order 2); the second-order coefficient polynomials on the boxes
  if ((rc = eval_level_prepared(R.QF, S, dom, fcl, fch, nullptr, scratch, sb, st, P, 1))) return rc;
  if ((rc = eval_level_prepared(R.QD, S, dom, dl, dh, nullptr, scratch, sb, st, R.M.dp.data(), t2 ? 1 : 0)))
    return rc;
  if (t2 && (rc = eval_level_prepared(R.QH, S, dom, hl, hh, nullptr, scratch, sb, st, R.M.hp.data(), 0))) return rc;
  CsfView cv;
  memset(&cv, 0, sizeof cv);
  for (int l = 0; l < k; l++) {
    cv.idx[l] = S->idx[l];
    cv.ptr[l] = S->ptr[l];
    cv.n[l] = S->n[l];
  }
  const unsigned nb = (unsigned)((nl + 255) / 256);
  hipLaunchKernelGGL(k_leaf_labels, dim3(nb), dim3(256), 0, st, k, cv, labels);
  VX_CHECK_LAUNCH("k_leaf_labels");
  GridSet gs;
  memset(&gs, 0, sizeof gs);
  for (int i = 0; i < k; i++) {
    AxisGrid g;
    g.dlo = dom[2 * i];
    g.dhi = dom[2 * i + 1];
    g.ndlo = -g.dlo;
    g.ndhi = -g.dhi;
    g.level = S->level;
    g.centre = 0;
    gs.cell[i] = g;
    g.centre = 1;
    gs.centre[i] = g;
    g.centre = 2;
    gs.vertex[i] = g;
  }
  if (incl) {
    hipLaunchKernelGGL(k_t2_inclusion, dim3(nb), dim3(256), 0, st, k, np, nl, gs, (const int32_t*)labels,
                       (const double*)fcl, (const double*)fch, (const double*)dl, (const double*)dh,
                       (const double*)hl, (const double*)hh, incl);
    VX_CHECK_LAUNCH("k_t2_inclusion");
  } else if (t2) {
    hipLaunchKernelGGL(k_t2_combine, dim3(nb), dim3(256), 0, st, k, np, nl, gs, (const int32_t*)labels,
                       (const double*)fcl, (const double*)fch, (const double*)dl, (const double*)dh,
                       (const double*)hl, (const double*)hh, lo, hi, keep);
    VX_CHECK_LAUNCH("k_t2_combine");
  } else {
    hipLaunchKernelGGL(k_mv_combine, dim3(nb), dim3(256), 0, st, k, np, nl, gs, (const int32_t*)labels,
                       (const double*)fcl, (const double*)fch, (const double*)dl, (const double*)dh, lo, hi, keep);
    VX_CHECK_LAUNCH("k_mv_combine");
  }
  prof_stop(pr, st);
  return VX_OK;
}

constexpr int TM_MAX_TERMS = 256;  // C(k + m, m) for k <= 4, m <= TAYLOR_MAX_ORDER (6): at most 210

__device__ __forceinline__ int64_t dbinom_i(int n, int r) {
  int64_t v = 1;
  for (int i = 1; i <= r; i++) v = v * (n - r + i) / i;
  return v;
}

// ---------------------------------------------------------------------------
// Taylor form of any order m (the same definition; orders 1 and 2 have the
// dedicated paths above, which give the same bits).  In k variables the term
// of order j at c is sum_{|alpha| = j} (D^alpha F / alpha!) (x - c)^alpha.
// The coefficient polynomial of alpha has entry e = prod_i C(e_i + alpha_i,
// alpha_i) c_{e + alpha}, an exact integer (< 2^53) times the coefficient,
// rounded outward once.  The terms of orders 0..m-1 are evaluated at the
// centre enclosures, those of order m over the boxes, each set as systems of
// polynomials through Algorithm 2 on the level's CSF; then per box
//   T_m(F, B) = F(c) + sum_{t >= 1} T_t X_t,  X_t = prod_i W_i^alpha_i,
// W_i = B_i - c_i, the ranges of the powers multiplied over ascending i, the
// terms summed left to right: orders 1..m, each order's multi-indices as the
// non-decreasing index tuples i_1 <= ... <= i_j in lexicographic order.
// ---------------------------------------------------------------------------
struct TermTab {
  int8_t a[TM_MAX_TERMS][VX_KMAX];  // multi-index of term t (t = 0: F itself)
  int n;                             // terms of orders 0..m
  int ncentre;                       // terms of orders 0..m-1
  int order;
};

static void term_tab_rec(TermTab& T, int k, int j, int from, int8_t* alpha, int left) {
  if (left == 0) {
    for (int i = 0; i < VX_KMAX; i++) T.a[T.n][i] = i < k ? alpha[i] : 0;
    T.n++;
    return;
  }
  for (int i = from; i < k; i++) {
    alpha[i]++;
    term_tab_rec(T, k, j, i, alpha, left - 1);
    alpha[i]--;
  }
}

static TermTab term_tab(int k, int m) {
  TermTab T;
  memset(&T, 0, sizeof T);
  T.order = m;
  for (int j = 0; j <= m; j++) {
    if (j == m) T.ncentre = T.n;
    int8_t alpha[VX_KMAX] = {0, 0, 0, 0};
    term_tab_rec(T, k, j, 0, alpha, j);
  }
  return T;
}

// One thread per (polynomial, term t >= 1, cube entry).
__global__ void k_taylor_coef(DerivArgs a, int k, TermTab T, int64_t cube_max, double* __restrict__ olo,
                              double* __restrict__ ohi) {
  round_up_mode();
  const int nt = T.n - 1;
  const int p = blockIdx.y / nt, t = 1 + blockIdx.y % nt;
  const int side = a.side[p], d = a.d[p];
  int64_t total = 1;
  for (int j = 0; j < k; j++) total *= side;
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= total) return;
  int e[VX_KMAX] = {0, 0, 0, 0};
  int64_t q = f, stride = 1, shift = 0;
  int deg = 0, order = 0;
  bool inside = true;
  for (int j = k - 1; j >= 0; j--) {
    e[j] = (int)(q % side);
    q /= side;
    deg += e[j];
    order += T.a[t][j];
    shift += T.a[t][j] * stride;
    inside = inside && e[j] + T.a[t][j] < side;
    stride *= side;
  }
  double* lo = olo + (int64_t)blockIdx.y * cube_max;
  double* hi = ohi + (int64_t)blockIdx.y * cube_max;
  if (deg + order > d || !inside) {
    lo[f] = 0.0;
    hi[f] = 0.0;
    return;
  }
  double m = 1.0;  // prod_i C(e_i + alpha_i, alpha_i): exact (the host keeps C(d + m, m) < 2^53)
  for (int j = 0; j < k; j++) m *= (double)dbinom_i(e[j] + T.a[t][j], T.a[t][j]);
  const int64_t src = f + shift;
  const double cl = a.clo[p][src];
  const double ch = a.chi[p] ? a.chi[p][src] : cl;
  lo[f] = -opaque(m * opaque(-cl));  // RD(m * cl) = -RU(m * -cl)
  hi[f] = m * ch;
}

// Range of x^a over W = [lo, hi] with lo <= 0 <= hi (W = B_i - c_i always
// holds 0), held as (nlo, hi), in round-up mode: odd a gives
// [-RU(nlo^a), RU(hi^a)], even a gives [0, RU(max(nlo, hi)^a)]; the powers
// of the nonnegative bounds by repeated multiplication, left to right.
__device__ __forceinline__ double pow_ru(double v, int a) {
  double p = v;
  for (int i = 1; i < a; i++) p = p * v;
  return p;
}

__device__ __forceinline__ void pow_straddle(double wnl, double wh, int a, double& pnl, double& ph) {
  if (a == 1) {
    pnl = wnl;
    ph = wh;
  } else if (a & 1) {
    pnl = pow_ru(wnl, a);
    ph = pow_ru(wh, a);
  } else {
    pnl = 0.0;
    ph = pow_ru(fmax(wnl, wh), a);
  }
}

// T_m for every leaf and polynomial; keep (if given) is AND-ed with "0 in
// T_m(F_p, B) for every p" (NaN endpoints never exclude).  Layouts: fc
// (np x nleaf), centre terms ((p, t - 1) x nleaf for t = 1..ncentre-1), box
// terms ((p, t - ncentre) x nleaf).
__global__ void k_tm_combine(int k, int np, int64_t nleaf, GridSet gs, const int32_t* __restrict__ labels,
                             TermTab T, const double* __restrict__ fc_lo, const double* __restrict__ fc_hi,
                             const double* __restrict__ tc_lo, const double* __restrict__ tc_hi,
                             const double* __restrict__ tb_lo, const double* __restrict__ tb_hi,
                             double* __restrict__ lo, double* __restrict__ hi, uint8_t* __restrict__ keep) {
  round_up_mode();
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nleaf) return;
  double wnl[VX_KMAX], wh[VX_KMAX];
  for (int i = 0; i < k; i++) {
    double inl, ih, cnl, ch;
    const int32_t lab = labels[b * k + i];
    cell(gs.cell[i], lab, inl, ih);
    cell(gs.centre[i], lab, cnl, ch);
    wnl[i] = ch + inl;  // -RD(lo_i - chi_i) = RU(chi_i - lo_i)
    wh[i] = ih + cnl;   // RU(hi_i - clo_i)
  }
  const int ncm = T.ncentre - 1, nbx = T.n - T.ncentre;
  bool excl = false;
  for (int p = 0; p < np; p++) {
    double anl = -opaque(fc_lo[(int64_t)p * nleaf + b]);
    double ah = fc_hi[(int64_t)p * nleaf + b];
    for (int t = 1; t < T.n; t++) {
      double xnl = 0.0, xh = 0.0;
      bool first = true;
      for (int i = 0; i < k; i++) {
        const int a = T.a[t][i];
        if (a == 0) continue;
        double pnl, ph;
        pow_straddle(wnl[i], wh[i], a, pnl, ph);
        if (first) {
          xnl = pnl;
          xh = ph;
          first = false;
        } else {
          mul_add_sep(xnl, xh, cell_ops(pnl, ph, CLS_STRADDLE), 0.0, 0.0);  // X * P (+ 0: exact)
        }
      }
      const int64_t ti = t < T.ncentre ? ((int64_t)p * ncm + (t - 1)) * nleaf + b
                                       : ((int64_t)p * nbx + (t - T.ncentre)) * nleaf + b;
      const double* tl = t < T.ncentre ? tc_lo : tb_lo;
      const double* th = t < T.ncentre ? tc_hi : tb_hi;
      double tnl = -opaque(tl[ti]);
      double tt = th[ti];
      mul_add_sep(tnl, tt, cell_ops(xnl, xh, CLS_STRADDLE), anl, ah);  // T_t * X_t + acc
      anl = tnl;
      ah = tt;
    }
    const double l = -opaque(anl);
    lo[(int64_t)p * nleaf + b] = l;
    hi[(int64_t)p * nleaf + b] = ah;
    excl = excl || (l > 0.0) || (ah < 0.0);
  }
  if (keep && excl) keep[b] = 0;
}

// The term polynomials of a run (coefficient cube pointers null when only
// sizes are wanted): centre terms (p, t = 1..ncentre-1) and box terms
// (p, t = ncentre..n-1), each list cut into systems of at most VX_MAXPOLY.
struct TmPolys {
  TermTab T;
  std::vector<vx_poly> tc, tb;
  int64_t cube_max = 1;
};

static TmPolys tm_polys(const vx_poly* P, int np, int order, double* clo, double* chi) {
  TmPolys M;
  const int k = P[0].k;
  M.T = term_tab(k, order);
  for (int p = 0; p < np; p++) {
    int64_t cube = 1;
    for (int j = 0; j < k; j++) cube *= P[p].side;
    M.cube_max = cube > M.cube_max ? cube : M.cube_max;
  }
  for (int p = 0; p < np; p++)
    for (int t = 1; t < M.T.n; t++) {
      int j = 0;
      for (int i = 0; i < k; i++) j += M.T.a[t][i];
      vx_poly q;
      memset(&q, 0, sizeof q);
      q.k = k;
      q.degree = P[p].degree > j ? P[p].degree - j : 0;
      q.side = P[p].side;
      const int64_t slot = (int64_t)p * (M.T.n - 1) + (t - 1);
      q.c_lo = clo ? clo + slot * M.cube_max : nullptr;
      q.c_hi = chi ? chi + slot * M.cube_max : nullptr;
      (t < M.T.ncentre ? M.tc : M.tb).push_back(q);
    }
  return M;
}

static int nchunks(size_t n) { return (int)((n + VX_MAXPOLY - 1) / VX_MAXPOLY); }

struct TmRun {
  TmPolys M;
  Prepared QF;
  std::vector<Prepared> QC, QB;  // per chunk of the centre and box term systems
  double* clo = nullptr;
  double* chi = nullptr;
};

static size_t chunk_prepared_bytes(const std::vector<vx_poly>& v) {
  size_t b = 0;
  for (int c = 0; c < nchunks(v.size()); c++) {
    const int n = (int)std::min(v.size() - (size_t)c * VX_MAXPOLY, (size_t)VX_MAXPOLY);
    b += (prepared_bytes(v.data() + (size_t)c * VX_MAXPOLY, n) + 255) / 256 * 256;
  }
  return b;
}

static size_t tm_run_bytes(const vx_poly* P, int np, int order) {
  TmPolys M = tm_polys(P, np, order, nullptr, nullptr);
  const size_t cubes = (sizeof(double) * (size_t)M.cube_max * np * (M.T.n - 1) + 255) / 256 * 256;
  return 2 * cubes + (prepared_bytes(P, np) + 255) / 256 * 256 + chunk_prepared_bytes(M.tc) +
         chunk_prepared_bytes(M.tb) + 2048;
}

static int prepare_chunks(const std::vector<vx_poly>& v, char*& at, std::vector<Prepared>& out, hipStream_t st) {
  int rc;
  for (int c = 0; c < nchunks(v.size()); c++) {
    const int n = (int)std::min(v.size() - (size_t)c * VX_MAXPOLY, (size_t)VX_MAXPOLY);
    const size_t b = (prepared_bytes(v.data() + (size_t)c * VX_MAXPOLY, n) + 255) / 256 * 256;
    Prepared Q;
    if ((rc = prepare_polys(v.data() + (size_t)c * VX_MAXPOLY, n, at, b, &Q, st))) return rc;
    out.push_back(Q);
    at += b;
  }
  return VX_OK;
}

static int tm_run_prepare(const vx_poly* P, int np, int order, char* ws, size_t bytes, TmRun& R, hipStream_t st) {
  if (tm_run_bytes(P, np, order) > bytes) VX_FAIL(VX_ECAPACITY, "Taylor test: workspace too small");
  TmPolys M0 = tm_polys(P, np, order, nullptr, nullptr);
  const size_t cubes = (sizeof(double) * (size_t)M0.cube_max * np * (M0.T.n - 1) + 255) / 256 * 256;
  R.clo = reinterpret_cast<double*>(ws);
  R.chi = reinterpret_cast<double*>(ws + cubes);
  R.M = tm_polys(P, np, order, R.clo, R.chi);
  const int k = P[0].k;
  hipLaunchKernelGGL(k_taylor_coef, dim3((unsigned)((R.M.cube_max + 255) / 256), (unsigned)(np * (R.M.T.n - 1))),
                     dim3(256), 0, st, deriv_args(P, np), k, R.M.T, R.M.cube_max, R.clo, R.chi);
  VX_CHECK_LAUNCH("k_taylor_coef");
  char* at = ws + 2 * cubes;
  const size_t qf = (prepared_bytes(P, np) + 255) / 256 * 256;
  int rc;
  if ((rc = prepare_polys(P, np, at, qf, &R.QF, st))) return rc;
  at += qf;
  if ((rc = prepare_chunks(R.M.tc, at, R.QC, st))) return rc;
  if ((rc = prepare_chunks(R.M.tb, at, R.QB, st))) return rc;
  return VX_OK;
}

static size_t tm_scratch_bytes(const vx_poly* P, int np, const TmPolys& M, const vx_csf* S) {
  size_t e = eval_level_bytes(P, np, S);
  for (const std::vector<vx_poly>* v : {&M.tc, &M.tb})
    for (int c = 0; c < nchunks(v->size()); c++) {
      const int n = (int)std::min(v->size() - (size_t)c * VX_MAXPOLY, (size_t)VX_MAXPOLY);
      const size_t b = eval_level_bytes(v->data() + (size_t)c * VX_MAXPOLY, n, S);
      e = b > e ? b : e;
    }
  return e;
}

static size_t tm_level_bytes(const vx_poly* P, int np, const TmPolys& M, const vx_csf* S) {
  const int k = S->k;
  const int64_t nl = S->n[k - 1];
  auto r = [](size_t b) { return (b + 255) / 256 * 256; };
  return r(sizeof(double) * np * nl) * 2 + r(sizeof(double) * M.tc.size() * nl + 8) * 2 +
         r(sizeof(double) * M.tb.size() * nl + 8) * 2 + r(sizeof(int32_t) * k * nl) + tm_scratch_bytes(P, np, M, S) +
         256;
}

static int eval_chunks(const std::vector<Prepared>& Q, const std::vector<vx_poly>& v, const vx_csf* S,
                       const double* dom, double* lo, double* hi, char* scratch, size_t sb, hipStream_t st,
                       int centre) {
  const int64_t nl = S->n[S->k - 1];
  int rc;
  for (size_t c = 0; c < Q.size(); c++) {
    const size_t off = c * VX_MAXPOLY;
    if ((rc = eval_level_prepared(Q[c], S, dom, lo + off * nl, hi + off * nl, nullptr, scratch, sb, st,
                                  v.data() + off, centre)))
      return rc;
  }
  return VX_OK;
}

static int tm_level(const vx_poly* P, int np, const TmRun& R, const vx_csf* S, const double* dom, double* lo,
                    double* hi, uint8_t* keep, char* ws, size_t bytes, hipStream_t st) {
  const int k = S->k;
  const int64_t nl = S->n[k - 1];
  if (nl == 0) return VX_OK;
  Arena A;
  A.base = ws;
  A.size = bytes;
  double* fcl = A.take<double>((size_t)np * nl);
  double* fch = A.take<double>((size_t)np * nl);
  double* tcl = A.take<double>(R.M.tc.size() * nl + 1);
  double* tch = A.take<double>(R.M.tc.size() * nl + 1);
  double* tbl = A.take<double>(R.M.tb.size() * nl + 1);
  double* tbh = A.take<double>(R.M.tb.size() * nl + 1);
  int32_t* labels = A.take<int32_t>((size_t)k * nl);
  const size_t sb = tm_scratch_bytes(P, np, R.M, S);
  char* scratch = A.take<char>(sb);
  if (A.overflow) VX_FAIL(VX_ECAPACITY, "Taylor test: workspace of %zu bytes is too small", bytes);
  const int pr = prof_start("taylor_m", (double)nl, st);
  int rc;
  // F and the terms of orders 1..m-1 at the centres, the order-m terms on the boxes
  if ((rc = eval_level_prepared(R.QF, S, dom, fcl, fch, nullptr, scratch, sb, st, P, 1))) return rc;
  if ((rc = eval_chunks(R.QC, R.M.tc, S, dom, tcl, tch, scratch, sb, st, 1))) return rc;
  if ((rc = eval_chunks(R.QB, R.M.tb, S, dom, tbl, tbh, scratch, sb, st, 0))) return rc;
  CsfView cv;
  memset(&cv, 0, sizeof cv);
  for (int l = 0; l < k; l++) {
    cv.idx[l] = S->idx[l];
    cv.ptr[l] = S->ptr[l];
    cv.n[l] = S->n[l];
  }
  const unsigned nb = (unsigned)((nl + 255) / 256);
  hipLaunchKernelGGL(k_leaf_labels, dim3(nb), dim3(256), 0, st, k, cv, labels);
  VX_CHECK_LAUNCH("k_leaf_labels");
  GridSet gs;
  memset(&gs, 0, sizeof gs);
  for (int i = 0; i < k; i++) {
    AxisGrid g;
    g.dlo = dom[2 * i];
    g.dhi = dom[2 * i + 1];
    g.ndlo = -g.dlo;
    g.ndhi = -g.dhi;
    g.level = S->level;
    g.centre = 0;
    gs.cell[i] = g;
    g.centre = 1;
    gs.centre[i] = g;
    g.centre = 2;
    gs.vertex[i] = g;
  }
  hipLaunchKernelGGL(k_tm_combine, dim3(nb), dim3(256), 0, st, k, np, nl, gs, (const int32_t*)labels, R.M.T,
                     (const double*)fcl, (const double*)fch, (const double*)tcl, (const double*)tch,
                     (const double*)tbl, (const double*)tbh, lo, hi, keep);
  VX_CHECK_LAUNCH("k_tm_combine");
  prof_stop(pr, st);
  return VX_OK;
}

size_t mv_workspace_bytes(const vx_poly* P, int np, const vx_csf* S, int order) {
  if (order >= 3) {
    TmPolys M = tm_polys(P, np, order, nullptr, nullptr);
    return (tm_run_bytes(P, np, order) + 255) / 256 * 256 + tm_level_bytes(P, np, M, S) + 512;
  }
  MvPolys M = mv_polys(P, np, order, nullptr, nullptr, nullptr, nullptr);
  return mv_run_bytes(P, np, order) + mv_level_bytes(P, np, M, S) + 512;
}

int mv_impl(const vx_poly* P, int np, const vx_csf* S, const double* dom, double* lo, double* hi, uint8_t* keep,
            void* ws, size_t ws_bytes, hipStream_t st, int order, uint8_t* incl) {
  if (S->n[S->k - 1] == 0) return VX_OK;
  if (order >= 3) {
    const size_t rb = (tm_run_bytes(P, np, order) + 255) / 256 * 256;
    if (rb > ws_bytes) VX_FAIL(VX_ECAPACITY, "Taylor test: workspace too small");
    TmRun R;
    int rc;
    if ((rc = tm_run_prepare(P, np, order, reinterpret_cast<char*>(ws), rb, R, st))) return rc;
    return tm_level(P, np, R, S, dom, lo, hi, keep, reinterpret_cast<char*>(ws) + rb, ws_bytes - rb, st);
  }
  const size_t rb = (mv_run_bytes(P, np, order) + 255) / 256 * 256;
  if (rb > ws_bytes) VX_FAIL(VX_ECAPACITY, "Taylor test: workspace too small");
  MvRun R;
  int rc;
  if ((rc = mv_run_prepare(P, np, order, reinterpret_cast<char*>(ws), rb, R, st))) return rc;
  return mv_level(P, np, R, S, dom, lo, hi, keep, reinterpret_cast<char*>(ws) + rb, ws_bytes - rb, st, incl);
}

// Run-level interface for run_subdivision: the tables are built once.
size_t mv_run_workspace(const vx_poly* P, int np, int order) {
  if (order >= 3) return (tm_run_bytes(P, np, order) + 255) / 256 * 256;
  return (mv_run_bytes(P, np, order) + 255) / 256 * 256;
}

size_t mv_level_workspace(const vx_poly* P, int np, const vx_csf* S, int order) {
  if (order >= 3) {
    TmPolys M = tm_polys(P, np, order, nullptr, nullptr);
    return tm_level_bytes(P, np, M, S);
  }
  MvPolys M = mv_polys(P, np, order, nullptr, nullptr, nullptr, nullptr);
  return mv_level_bytes(P, np, M, S);
}

struct MvRunHandle {
  int order = 1;
  MvRun R;
  TmRun T;
};

void* mv_run_begin(const vx_poly* P, int np, void* ws, size_t bytes, hipStream_t st, int* rc, int order) {
  MvRunHandle* h = new MvRunHandle;
  h->order = order;
  *rc = order >= 3 ? tm_run_prepare(P, np, order, reinterpret_cast<char*>(ws), bytes, h->T, st)
                   : mv_run_prepare(P, np, order, reinterpret_cast<char*>(ws), bytes, h->R, st);
  if (*rc) {
    delete h;
    return nullptr;
  }
  return h;
}

int mv_run_level(void* handle, const vx_poly* P, int np, const vx_csf* S, const double* dom, double* lo, double* hi,
                 uint8_t* keep, void* ws, size_t bytes, hipStream_t st) {
  const MvRunHandle* h = reinterpret_cast<const MvRunHandle*>(handle);
  if (h->order >= 3) return tm_level(P, np, h->T, S, dom, lo, hi, keep, reinterpret_cast<char*>(ws), bytes, st);
  return mv_level(P, np, h->R, S, dom, lo, hi, keep, reinterpret_cast<char*>(ws), bytes, st);
}

void mv_run_end(void* handle) { delete reinterpret_cast<MvRunHandle*>(handle); }

// ---------------------------------------------------------------------------
// Inclusion criterion C1 (Sec. 3.2): F on the 2^k vertices of every box; the
// box is certified to meet F = 0 when one vertex enclosure is > 0 and another
// < 0 (intermediate value theorem along the box's edges).  The vertices of all
// boxes are grid points, evaluated once each by Algorithm 2 on the degenerate
// vertex enclosures of their own CSF; every box then reads its vertices'
// values through a corner table.
//
// The vertex CSF is built in closed form from the box CSF, depth by depth,
// without listing or sorting vertex tuples.  A vertex prefix (v_0 .. v_l) is
// a corner prefix of the box prefixes (v_0 - b_0 .. v_l - b_l), b_i in {0, 1}:
// its "sources", at most 2^(l+1) box CSF nodes, indexed by beta = the bits
// b_0 .. b_l (b_0 most significant).  The children of a vertex node are the
// union over its sources s of {c, c + 1} for the children labels c of s (a
// counting pass, a scan, a writing pass, one wave per vertex node).  The child w's sources are the children c = w - b of the
// parent's sources, at beta' = 2 beta + b.  At the last depth beta' is the
// corner index m of box c (bit k-1-j of m = the offset on axis j), so the
// writing pass fills corner[m * N + c] (N boxes; corner-major, so that the
// vertices of neighbouring boxes are stored side by side) with the vertex's
// index: every corner of every box is written exactly once.  The labels
// come out sorted and without repeats, so the CSF is the one of the sorted
// vertex set.
// ---------------------------------------------------------------------------

struct VtxJob {
  int k;
  CsfView S;                 // the boxes
  int32_t* vidx[VX_KMAX];    // the vertex CSF
  int32_t* vptr[VX_KMAX];
  int32_t* src[VX_KMAX];     // src[l][v * 2^(l+1) + beta], l < k - 1 (-1: none)
  int32_t* corner;           // corner[m * nbox + b]: vertex of corner m of box b
  int64_t nbox;
  int64_t* cnt;              // children per vertex node of the depth being built
  int64_t* vn;               // vertex nodes per depth (device)
};

// Store vertex o of depth l with its sources (nsrc = 2^(l+1) of them).
__device__ __forceinline__ void vtx_store(const VtxJob& J, int l, int64_t o, int32_t w, const int32_t* srcs,
                                          int nsrc) {
  J.vidx[l][o] = w;
  if (l == J.k - 1) {
    for (int b = 0; b < nsrc; b++)
      if (srcs[b] >= 0) J.corner[(int64_t)b * J.nbox + srcs[b]] = (int32_t)o;
  } else {
    for (int b = 0; b < nsrc; b++) J.src[l][o * nsrc + b] = srcs[b];
  }
}

// Depth 0: box node i (label a) gives vertex a, unless a - 1 is the box
// label before it (then a is that node's a + 1), and vertex a + 1.
__global__ void k_vtx0(VtxJob J, int write, const int64_t* __restrict__ off) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = J.S.n[0];
  if (i >= n) return;
  const int32_t* idx = J.S.idx[0];
  const int32_t a = idx[i];
  const bool lead = i == 0 || idx[i - 1] != a - 1;
  if (!write) {
    J.cnt[i] = lead ? 2 : 1;
    return;
  }
  int64_t o = off[i];
  if (lead) {
    const int32_t s[2] = {(int32_t)i, -1};
    vtx_store(J, 0, o++, a, s, 2);
  }
  const int32_t s[2] = {(i + 1 < n && idx[i + 1] == a + 1) ? (int32_t)(i + 1) : -1, (int32_t)i};
  vtx_store(J, 0, o, a + 1, s, 2);
}

// The children of vertex node v (depth L) by a sequential merge of its
// 2^(L+1) source runs, each run giving c and c + 1 for its labels c; returns
// their number and, with `write`, stores them from index o on.
template <int L>
__device__ int64_t vtx_merge_node(const VtxJob& J, int64_t v, bool write, int64_t o) {
  constexpr int NS = 1 << (L + 1);
  const int32_t* cidx = J.S.idx[L + 1];
  const int32_t* sptr = J.S.ptr[L];
  constexpr int32_t NONE = 0x7fffffff;
  int64_t p[NS], e[NS];
  int32_t c[NS];
  int ph[NS];
#pragma unroll
  for (int b = 0; b < NS; b++) {
    const int32_t s = J.src[L][v * NS + b];
    p[b] = s >= 0 ? sptr[s] : 0;
    e[b] = s >= 0 ? sptr[s + 1] : 0;
    c[b] = p[b] < e[b] ? cidx[p[b]] : NONE;
    ph[b] = 0;
  }
  int64_t count = 0;
  while (true) {
    int32_t w = NONE;
#pragma unroll
    for (int b = 0; b < NS; b++)
      if (c[b] != NONE && c[b] + ph[b] < w) w = c[b] + ph[b];
    if (w == NONE) break;
    int32_t srcs[2 * NS];
#pragma unroll
    for (int b = 0; b < 2 * NS; b++) srcs[b] = -1;
#pragma unroll
    for (int b = 0; b < NS; b++)
      while (c[b] != NONE && c[b] + ph[b] == w) {  // at most twice: (c, +1) and (c + 1, +0)
        srcs[2 * b + ph[b]] = (int32_t)p[b];
        if (ph[b] == 0) {
          ph[b] = 1;
        } else {
          ph[b] = 0;
          p[b]++;
          c[b] = p[b] < e[b] ? cidx[p[b]] : NONE;
        }
      }
    if (write) vtx_store(J, L + 1, o++, w, srcs, 2 * NS);
    count++;
  }
  return count;
}

// Depth L + 1 under every vertex node of depth L, one wave (one workgroup of
// 64) per node.  The node's children lie in the label window [lo, hi] (lo the
// smallest first label of its source runs, hi the largest last label + 1);
// when the window spans at most VTX_WORDS 64-bit words, each source run is
// set as a bitmap over the window in LDS (run b: bit x for label lo + x), the
// children are the set bits of U = OR_b (B_b | B_b << 1), and the source of
// child w at (b, d) is the run's element of label w - d, whose index is its
// rank in B_b.  Lane j owns word j.  Wider windows take the sequential merge
// on lane 0.
constexpr int VTX_WORDS = 64;

template <int L>
__global__ __launch_bounds__(64) void k_vtx_merge(VtxJob J, int write, const int64_t* __restrict__ off) {
  constexpr int NS = 1 << (L + 1);
  __shared__ uint64_t bits[NS][VTX_WORDS];
  __shared__ int64_t rank[NS][VTX_WORDS];  // set bits of B_b in the words before word j
  const int64_t v = blockIdx.x;
  const int64_t nv = J.vn[L];
  if (v >= nv) return;  // uniform: one wave per workgroup
  const int lane = threadIdx.x;
  const int32_t* cidx = J.S.idx[L + 1];
  const int32_t* sptr = J.S.ptr[L];
  int64_t p[NS], e[NS];
  int32_t lo = 0x7fffffff, hi = -1;
#pragma unroll
  for (int b = 0; b < NS; b++) {
    const int32_t s = J.src[L][v * NS + b];
    p[b] = s >= 0 ? sptr[s] : 0;
    e[b] = s >= 0 ? sptr[s + 1] : 0;
    if (p[b] < e[b]) {
      lo = min(lo, cidx[p[b]]);
      hi = max(hi, cidx[e[b] - 1] + 1);
    }
  }
  const int64_t o0 = write ? off[v] : 0;
  if (write) {
    if (lane == 0) J.vptr[L][v] = (int32_t)o0;
    if (lane == 0 && v == nv - 1) J.vptr[L][nv] = (int32_t)off[nv];
  }
  const int64_t width = (int64_t)hi - lo + 1;
  if (width > 64 * VTX_WORDS) {
    if (lane == 0) {
      const int64_t n = vtx_merge_node<L>(J, v, write != 0, o0);
      if (!write) J.cnt[v] = n;
    }
    return;
  }
  const int nw = (int)((width + 63) / 64);
#pragma unroll
  for (int b = 0; b < NS; b++) bits[b][lane] = 0;
  __syncthreads();
#pragma unroll
  for (int b = 0; b < NS; b++)
    for (int64_t i = p[b] + lane; i < e[b]; i += 64) {
      const int x = cidx[i] - lo;
      atomicOr(reinterpret_cast<unsigned long long*>(&bits[b][x >> 6]), 1ull << (x & 63));
    }
  __syncthreads();
  uint64_t u = 0;
  if (lane < nw) {
#pragma unroll
    for (int b = 0; b < NS; b++) u |= bits[b][lane] | (bits[b][lane] << 1) | (lane > 0 ? bits[b][lane - 1] >> 63 : 0);
  }
  const int64_t cnt = __popcll(u);
  if (!write) {
    int64_t tot = cnt;
    for (int d = 32; d >= 1; d >>= 1) tot += __shfl_xor(tot, d, 64);
    if (lane == 0) J.cnt[v] = tot;
    return;
  }
  // exclusive prefix over the lanes: of the children, and of each run's bits
  auto excl_scan = [&](int64_t x) {
    int64_t inc = x;
    for (int d = 1; d < 64; d <<= 1) {
      const int64_t y = __shfl_up(inc, d, 64);
      if (lane >= d) inc += y;
    }
    return inc - x;
  };
  __shared__ uint64_t uw[VTX_WORDS];
  __shared__ int32_t upre[VTX_WORDS + 1];
  const int64_t pre = excl_scan(cnt);
  uw[lane] = u;
  upre[lane] = (int32_t)pre;
  if (lane == 63) upre[64] = (int32_t)(pre + cnt);
#pragma unroll
  for (int b = 0; b < NS; b++) rank[b][lane] = excl_scan(__popcll(bits[b][lane]));
  __syncthreads();
  // child t of the node goes to lane t mod 64 (so that lanes share the
  // work and neighbouring lanes store neighbouring entries): its word is the
  // last j with upre[j] <= t, its bit the (t - upre[j])-th set bit of word j
  const int total = upre[64];
  for (int t = lane; t < total; t += 64) {
    int j = 0;
    for (int step = 32; step >= 1; step >>= 1)
      if (upre[j + step] <= t) j += step;
    uint64_t wv = uw[j];
    int r = t - upre[j], x = 0;
    for (int sh = 32; sh >= 1; sh >>= 1) {
      const int c = __popcll(wv & ((1ull << sh) - 1));
      if (r >= c) {
        r -= c;
        wv >>= sh;
        x += sh;
      }
    }
    const int pos = j * 64 + x;  // window position of the child
    const int64_t o = o0 + t;
    int32_t srcs[2 * NS];
#pragma unroll
    for (int b = 0; b < NS; b++)
#pragma unroll
      for (int d = 0; d < 2; d++) {
        const int y = pos - d;  // window position of label w - d
        int32_t sv = -1;
        if (y >= 0) {
          const uint64_t wb = bits[b][y >> 6];
          if ((wb >> (y & 63)) & 1)
            sv = (int32_t)(p[b] + rank[b][y >> 6] + __popcll(wb & ((1ull << (y & 63)) - 1)));
        }
        srcs[2 * b + d] = sv;
      }
    vtx_store(J, L + 1, o, lo + pos, srcs, 2 * NS);
  }
}

struct VtxCountLoader {
  const int64_t* c;
  __device__ int64_t operator()(int64_t i) const { return c[i]; }
};

// incl[p * nleaf + b] = 1 when some vertex of box b has a lower bound > 0 and
// another an upper bound < 0 for F_p (NaN bounds certify nothing).
__global__ void k_c1_flags(int k, int np, int64_t nleaf, const int32_t* __restrict__ corner, int64_t nv,
                           const double* __restrict__ vlo, const double* __restrict__ vhi,
                           uint8_t* __restrict__ incl) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nleaf) return;
  const int nc = 1 << k;
  uint64_t pos = 0, neg = 0;
  for (int m = 0; m < nc; m++) {
    const int64_t q = corner[(int64_t)m * nleaf + b];
    for (int p = 0; p < np; p++) {
      if (vlo[(int64_t)p * nv + q] > 0.0) pos |= 1ull << p;
      if (vhi[(int64_t)p * nv + q] < 0.0) neg |= 1ull << p;
    }
  }
  for (int p = 0; p < np; p++) incl[(int64_t)p * nleaf + b] = (uint8_t)(((pos & neg) >> p) & 1);
}

struct InclPlan {
  VtxJob J;
  vx_csf V;
  int64_t* off = nullptr;
  int64_t* tiles = nullptr;
  int64_t cmax = 1;
  double* vlo = nullptr;
  double* vhi = nullptr;
  char* eval_ws = nullptr;
  size_t eval_bytes = 0;
};

// Vertex CSF capacities: depth l holds at most min((2^level + 1)^(l+1),
// 2^(l+1) N_l) nodes (each box node is a source of at most 2^(l+1) vertex
// nodes, each vertex node has a source).
static void plan_inclusion(Arena& A, InclPlan& I, const vx_poly* P, int np, const vx_csf* S) {
  const int k = S->k;
  const int64_t n = S->n[k - 1];
  const int64_t side = ((int64_t)1 << S->level) + 1;
  memset(&I.V, 0, sizeof I.V);
  memset(&I.J, 0, sizeof I.J);
  I.V.k = k;
  I.V.level = S->level;
  I.J.k = k;
  int64_t grid = 1;
  I.cmax = 1;
  for (int l = 0; l < k; l++) {
    grid = grid > ((int64_t)1 << 40) ? grid : grid * side;
    const int64_t b = S->n[l] << (l + 1);
    I.V.cap[l] = grid < b ? grid : b;
    I.V.n[l] = I.V.cap[l];
    I.cmax = I.V.cap[l] > I.cmax ? I.V.cap[l] : I.cmax;
  }
  for (int l = 0; l < k; l++) {
    I.V.idx[l] = A.take<int32_t>((size_t)I.V.cap[l] + 1);
    if (l + 1 < k) {
      I.V.ptr[l] = A.take<int32_t>((size_t)I.V.cap[l] + 1);
      I.J.src[l] = A.take<int32_t>((size_t)I.V.cap[l] << (l + 1));
    }
    I.J.vidx[l] = I.V.idx[l];
    I.J.vptr[l] = I.V.ptr[l];
  }
  I.J.corner = A.take<int32_t>((size_t)(n > 0 ? n : 1) << k);
  I.J.cnt = A.take<int64_t>((size_t)I.cmax + 1);
  I.J.vn = A.take<int64_t>(VX_KMAX);
  I.off = A.take<int64_t>((size_t)I.cmax + 1);
  I.tiles = A.take<int64_t>(scan_tiles(I.cmax));
  I.vlo = A.take<double>((size_t)np * I.V.cap[k - 1]);
  I.vhi = A.take<double>((size_t)np * I.V.cap[k - 1]);
  // the vertex counts are known only after the build: plan for their bounds
  I.eval_bytes = prepared_bytes(P, np) + eval_level_bytes_bound(P, np, &I.V) + 256;
  I.eval_ws = A.take<char>(I.eval_bytes);
}

size_t inclusion_workspace_bytes(const vx_poly* P, int np, const vx_csf* S) {
  Arena A;
  InclPlan I;
  plan_inclusion(A, I, P, np, S);
  return A.off + 256;
}

int inclusion_impl(const vx_poly* P, int np, const vx_csf* S, const double* dom, uint8_t* incl, void* ws,
                   size_t ws_bytes, hipStream_t st) {
  const int k = S->k;
  const int64_t n = S->n[k - 1];
  if (n == 0) return VX_OK;
  if (S->level > 29) VX_FAIL(VX_EUNSUPPORTED, "inclusion test: level %d exceeds the int32 vertex labels", S->level);
  Arena A;
  A.base = reinterpret_cast<char*>(ws);
  A.size = ws_bytes;
  InclPlan I;
  plan_inclusion(A, I, P, np, S);
  if (A.overflow) VX_FAIL(VX_ECAPACITY, "inclusion test: workspace of %zu bytes is too small", ws_bytes);
  const int pr = prof_start("inclusion", (double)n, st);
  VtxJob& J = I.J;
  J.nbox = n;
  for (int l = 0; l < k; l++) {
    J.S.idx[l] = S->idx[l];
    J.S.ptr[l] = S->ptr[l];
    J.S.n[l] = S->n[l];
  }
  // depth 0
  const int64_t n0 = S->n[0];
  hipLaunchKernelGGL(k_vtx0, dim3((unsigned)((n0 + 255) / 256)), dim3(256), 0, st, J, 0, (const int64_t*)nullptr);
  scan_exclusive(VtxCountLoader{J.cnt}, (const int64_t*)nullptr, n0, I.off, J.vn, I.tiles, st);
  hipLaunchKernelGGL(k_vtx0, dim3((unsigned)((n0 + 255) / 256)), dim3(256), 0, st, J, 1, (const int64_t*)I.off);
  VX_CHECK_LAUNCH("k_vtx0");
  // depths 1 .. k-1; grids from the capacities, counts read on the device
  for (int l = 0; l + 1 < k; l++) {
    const dim3 grid((unsigned)I.V.cap[l]);  // one wave per vertex node
    auto merge = [&](int write) {
      switch (l) {
        case 0: hipLaunchKernelGGL(k_vtx_merge<0>, grid, dim3(64), 0, st, J, write, (const int64_t*)I.off); break;
        case 1: hipLaunchKernelGGL(k_vtx_merge<1>, grid, dim3(64), 0, st, J, write, (const int64_t*)I.off); break;
        default: hipLaunchKernelGGL(k_vtx_merge<2>, grid, dim3(64), 0, st, J, write, (const int64_t*)I.off); break;
      }
    };
    merge(0);
    scan_exclusive(VtxCountLoader{J.cnt}, (const int64_t*)(J.vn + l), I.V.cap[l], I.off, J.vn + l + 1, I.tiles, st);
    merge(1);
    VX_CHECK_LAUNCH("k_vtx_merge");
  }
  int64_t vn[VX_KMAX] = {0, 0, 0, 0};
  VX_HIP(hipMemcpyAsync(vn, J.vn, sizeof(int64_t) * k, hipMemcpyDeviceToHost, st));
  VX_HIP(hipStreamSynchronize(st));
  for (int l = 0; l < k; l++) {
    if (vn[l] > I.V.cap[l]) VX_FAIL(VX_EHIP, "inclusion test: vertex depth %d holds %lld nodes, over its bound %lld", l,
                                    (long long)vn[l], (long long)I.V.cap[l]);
    I.V.n[l] = vn[l];
  }
  I.V.level = S->level;
  int rc;
  if ((rc = eval_level_impl(P, np, &I.V, dom, I.vlo, I.vhi, nullptr, I.eval_ws, I.eval_bytes, st, 2))) return rc;
  hipLaunchKernelGGL(k_c1_flags, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, k, np, n,
                     (const int32_t*)J.corner, vn[k - 1], (const double*)I.vlo, (const double*)I.vhi, incl);
  VX_CHECK_LAUNCH("k_c1_flags");
  prof_stop(pr, st);
  return VX_OK;
}

// ---------------------------------------------------------------------------
// Newton interval inclusion test for a square system (Sec. 3.2, inclusion
// criterion for several polynomials), in Krawczyk's form:
//   K(B) = c - Y F(c) + (I - Y S)(B - c),   Y = (mid S)^-1,
// S the slope matrix: S_ij enclosed by dF_i/dx_j on the box with the
// variables 1..j free and j+1..k at the centre (Algorithm 2 with cell
// enclosures on the first j+1 axes and centre enclosures on the others).
// K(B) inside B means x - Y F(x) maps B into itself, so (Brouwer) F has a
// zero in B.  Y is computed in round-to-nearest by one kernel, K in outward
// arithmetic by another (each kernel keeps one rounding mode).
// ---------------------------------------------------------------------------

// Y = (mid S)^-1 per box: mid = (lo + hi) * 0.5, Gauss-Jordan with partial
// pivoting (first largest |pivot|), rows swapped in both matrices, the
// pivot row divided by the pivot, then row r -= f * pivot row for every
// other row; a zero (or NaN) pivot leaves ok = 0.  S_ij sits at
// ((j * k + i) * nleaf + b), Y_ij is written at ((i * k + j) * nleaf + b).
__global__ void k_newton_y(int k, int64_t nleaf, const double* __restrict__ s_lo, const double* __restrict__ s_hi,
                           double* __restrict__ Y, uint8_t* __restrict__ ok) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nleaf) return;
  double A[VX_KMAX][VX_KMAX], Z[VX_KMAX][VX_KMAX];
  for (int i = 0; i < k; i++)
    for (int j = 0; j < k; j++) {
      const int64_t e = ((int64_t)j * k + i) * nleaf + b;
      A[i][j] = (s_lo[e] + s_hi[e]) * 0.5;
      Z[i][j] = i == j ? 1.0 : 0.0;
    }
  int good = 1;
  for (int col = 0; col < k && good; col++) {
    int piv = col;
    for (int r = col + 1; r < k; r++)
      if (fabs(A[r][col]) > fabs(A[piv][col])) piv = r;
    if (!(A[piv][col] != 0.0)) {
      good = 0;
      break;
    }
    if (piv != col)
      for (int j = 0; j < k; j++) {
        double t = A[col][j];
        A[col][j] = A[piv][j];
        A[piv][j] = t;
        t = Z[col][j];
        Z[col][j] = Z[piv][j];
        Z[piv][j] = t;
      }
    const double p = A[col][col];
    for (int j = 0; j < k; j++) {
      A[col][j] = A[col][j] / p;
      Z[col][j] = Z[col][j] / p;
    }
    for (int r = 0; r < k; r++) {
      if (r == col) continue;
      const double f = A[r][col];
      for (int j = 0; j < k; j++) {
        A[r][j] = A[r][j] - f * A[col][j];
        Z[r][j] = Z[r][j] - f * Z[col][j];
      }
    }
  }
  for (int i = 0; i < k; i++)
    for (int j = 0; j < k; j++) Y[((int64_t)i * k + j) * nleaf + b] = good ? Z[i][j] : 0.0;
  ok[b] = (uint8_t)good;
}

// Point y times interval (xnl, xh), in (nlo, hi): the product rule with the
// degenerate interval [y, y].
__device__ __forceinline__ void point_times(double y, double xnl, double xh, double& rnl, double& rh) {
  rnl = xnl;
  rh = xh;
  mul_add_sep(rnl, rh, cell_ops(opaque(-y), y, CLS_STRADDLE), 0.0, 0.0);
}

// K(B) per box in outward arithmetic and the test K inside the inner box
// [upper end of the lower vertex enclosure, lower end of the upper one]
// (inside the true box): Yf_i = sum_j Y_ij F_j(c), K_i = (c_i - Yf_i) +
// sum_j A_ij W_j with A_ij = delta_ij - sum_l Y_il S_lj, sums in ascending
// index order, W_j = B_j - c_j.
__global__ void k_newton_k(int k, int64_t nleaf, GridSet gs, const int32_t* __restrict__ labels,
                           const double* __restrict__ fc_lo, const double* __restrict__ fc_hi,
                           const double* __restrict__ s_lo, const double* __restrict__ s_hi,
                           const double* __restrict__ Y, const uint8_t* __restrict__ ok, uint8_t* __restrict__ incl,
                           double* __restrict__ kout) {
  round_up_mode();
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nleaf) return;
  double cnl[VX_KMAX], ch[VX_KMAX], in_lo[VX_KMAX], in_hi[VX_KMAX];
  CellOps W[VX_KMAX];
  for (int a = 0; a < k; a++) {
    double inl, ih, vnl, vh;
    const int32_t lab = labels[b * k + a];
    cell(gs.cell[a], lab, inl, ih);
    cell(gs.centre[a], lab, cnl[a], ch[a]);
    W[a] = cell_ops(ch[a] + inl, ih + cnl[a], CLS_STRADDLE);
    cell(gs.vertex[a], lab, vnl, vh);
    in_lo[a] = vh;  // upper end of the lower vertex
    cell(gs.vertex[a], lab + 1, vnl, vh);
    in_hi[a] = -opaque(vnl);  // lower end of the upper vertex
  }
  const bool good = ok[b] != 0;
  bool inside = good;
  for (int i = 0; i < k; i++) {
    double knl = 0.0, kh = 0.0;
    if (good) {
      double ynl = 0.0, yh = 0.0;
      for (int j = 0; j < k; j++) {
        const double y = Y[((int64_t)i * k + j) * nleaf + b];
        double pnl, ph;
        point_times(y, -opaque(fc_lo[(int64_t)j * nleaf + b]), fc_hi[(int64_t)j * nleaf + b], pnl, ph);
        if (j == 0) {
          ynl = pnl;
          yh = ph;
        } else {
          ynl = ynl + pnl;
          yh = yh + ph;
        }
      }
      knl = cnl[i] + yh;  // c_i - Yf_i
      kh = ch[i] + ynl;
      for (int j = 0; j < k; j++) {
        double anl = i == j ? -1.0 : opaque(-0.0), ah = i == j ? 1.0 : 0.0;
        for (int l = 0; l < k; l++) {
          const int64_t e = ((int64_t)j * k + l) * nleaf + b;  // S_lj
          double tnl, th;
          point_times(Y[((int64_t)i * k + l) * nleaf + b], -opaque(s_lo[e]), s_hi[e], tnl, th);
          anl = anl + th;  // a - t
          ah = ah + tnl;
        }
        mul_add_sep(anl, ah, W[j], knl, kh);  // A_ij W_j + K_i
        knl = anl;
        kh = ah;
      }
      inside = inside && (-opaque(knl) >= in_lo[i]) && (kh <= in_hi[i]);
    }
    if (kout) {
      kout[(b * k + i) * 2] = -opaque(knl);
      kout[(b * k + i) * 2 + 1] = kh;
    }
  }
  incl[b] = (uint8_t)inside;
}

// ---------------------------------------------------------------------------
// Newton test for m < k polynomials (Sec. 3.2, inclusion criterion, last
// paragraph): the box is intersected with the plane through a point c of it
// spanned by the gradients at its centre, x = c + G y, and the square system
// phi(y) = F(c + G y) is tested on a cube Y = [-r, r]^m whose image fits the
// box.  c = the lower end of the centre enclosure, G (k x m) = the midpoints
// of the gradient enclosures at the centre, r = the largest power of two
// with s_j r <= min(c_j - lo_j, hi_j - c_j) for s_j = sum_l |G_jl| (rounded
// up, the room rounded down), and Krawczyk's operator
//   K(Y) = -M phi(0) + (I - M A) Y,   A = D G,   M = (mid(D) G)^-1,
// D the Jacobian enclosed on the box (so A encloses phi's Jacobian on Y),
// phi(0) enclosed by F on the centre enclosure.  K inside the open cube
// certifies a zero of phi in Y, hence of F in c + G Y, inside the box.
// G, mid(D) G and M are computed in round-to-nearest (one kernel), every
// enclosure outward (another).  Derivative enclosures sit at
// ((i * k + j) * nleaf + b), F_i at (i * nleaf + b).
// ---------------------------------------------------------------------------

// G (at ((j * m + l) * nleaf + b)) and M = (mid(D) G)^-1 (at ((i * m + l) *
// nleaf + b)) per box; Gauss-Jordan as in k_newton_y.
__global__ void k_span_m(int k, int m, int64_t nleaf, const double* __restrict__ gc_lo,
                         const double* __restrict__ gc_hi, const double* __restrict__ d_lo,
                         const double* __restrict__ d_hi, double* __restrict__ Gout, double* __restrict__ Mout,
                         uint8_t* __restrict__ ok) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nleaf) return;
  double G[VX_KMAX][VX_KMAX], A[VX_KMAX][VX_KMAX], Z[VX_KMAX][VX_KMAX];
  for (int j = 0; j < k; j++)
    for (int l = 0; l < m; l++) {
      const int64_t e = ((int64_t)l * k + j) * nleaf + b;
      G[j][l] = (gc_lo[e] + gc_hi[e]) * 0.5;
    }
  for (int i = 0; i < m; i++)
    for (int l = 0; l < m; l++) {
      double acc = 0.0;
      for (int j = 0; j < k; j++) {
        const int64_t e = ((int64_t)i * k + j) * nleaf + b;
        const double t = ((d_lo[e] + d_hi[e]) * 0.5) * G[j][l];
        acc = j == 0 ? t : acc + t;
      }
      A[i][l] = acc;
      Z[i][l] = i == l ? 1.0 : 0.0;
    }
  int good = 1;
  for (int col = 0; col < m && good; col++) {
    int piv = col;
    for (int r = col + 1; r < m; r++)
      if (fabs(A[r][col]) > fabs(A[piv][col])) piv = r;
    if (!(A[piv][col] != 0.0)) {
      good = 0;
      break;
    }
    if (piv != col)
      for (int j = 0; j < m; j++) {
        double t = A[col][j];
        A[col][j] = A[piv][j];
        A[piv][j] = t;
        t = Z[col][j];
        Z[col][j] = Z[piv][j];
        Z[piv][j] = t;
      }
    const double p = A[col][col];
    for (int j = 0; j < m; j++) {
      A[col][j] = A[col][j] / p;
      Z[col][j] = Z[col][j] / p;
    }
    for (int r = 0; r < m; r++) {
      if (r == col) continue;
      const double f = A[r][col];
      for (int j = 0; j < m; j++) {
        A[r][j] = A[r][j] - f * A[col][j];
        Z[r][j] = Z[r][j] - f * Z[col][j];
      }
    }
  }
  for (int j = 0; j < k; j++)
    for (int l = 0; l < m; l++) Gout[((int64_t)j * m + l) * nleaf + b] = G[j][l];
  for (int i = 0; i < m; i++)
    for (int l = 0; l < m; l++) Mout[((int64_t)i * m + l) * nleaf + b] = good ? Z[i][l] : 0.0;
  ok[b] = (uint8_t)good;
}

// The cube, A = D G, K and the test, in outward arithmetic.
__global__ void k_span_k(int k, int m, int64_t nleaf, GridSet gs, const int32_t* __restrict__ labels,
                         const double* __restrict__ fc_lo, const double* __restrict__ fc_hi,
                         const double* __restrict__ d_lo, const double* __restrict__ d_hi,
                         const double* __restrict__ Gm, const double* __restrict__ Mm,
                         const uint8_t* __restrict__ ok, uint8_t* __restrict__ incl, double* __restrict__ kout) {
  round_up_mode();
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nleaf) return;
  double G[VX_KMAX][VX_KMAX];
  for (int j = 0; j < k; j++)
    for (int l = 0; l < m; l++) G[j][l] = Gm[((int64_t)j * m + l) * nleaf + b];
  bool good = ok[b] != 0;
  // s_j r <= room_j on every axis with s_j > 0; r = 2^e
  int e = 0;
  bool have = false;
  double sj[VX_KMAX], room[VX_KMAX];
  for (int j = 0; j < k; j++) {
    double inl, ih, cnl, ch;
    const int32_t lab = labels[b * k + j];
    cell(gs.cell[j], lab, inl, ih);
    cell(gs.centre[j], lab, cnl, ch);
    const double c = opaque(-cnl);  // the lower end of the centre enclosure
    double s = fabs(G[j][0]);
    for (int l = 1; l < m; l++) s = s + fabs(G[j][l]);  // rounded up
    const double r1 = -opaque(cnl + opaque(-inl));  // RD(c - lo) = -RU(lo - c)
    const double r2 = -opaque(c + opaque(-ih));     // RD(hi - c) = -RU(c - hi)
    sj[j] = s;
    room[j] = r1 < r2 ? r1 : r2;
    if (!good || !(s > 0.0)) continue;
    if (!(room[j] > 0.0)) {
      good = false;
      continue;
    }
    const int ej = ilogb(room[j]) - ilogb(s);
    e = have ? (ej < e ? ej : e) : ej;
    have = true;
  }
  if (!have) good = false;
  if (good) {
    bool fits = true;
    for (int j = 0; j < k; j++)
      if (sj[j] > 0.0 && !(ldexp(sj[j], e) <= room[j])) fits = false;
    if (!fits) e -= 1;
  }
  const double r = good ? ldexp(1.0, e) : 0.0;
  const CellOps Ycube = cell_ops(r, r, CLS_STRADDLE);  // [-r, r]
  // A = D G (m x m intervals, (nlo, hi))
  double anl[VX_KMAX][VX_KMAX], ah[VX_KMAX][VX_KMAX];
  for (int q = 0; q < m; q++)
    for (int l = 0; l < m; l++) {
      double accn = 0.0, acch = 0.0;
      for (int j = 0; j < k; j++) {
        const int64_t ei = ((int64_t)q * k + j) * nleaf + b;
        double tnl, th;
        point_times(G[j][l], -opaque(d_lo[ei]), d_hi[ei], tnl, th);
        if (j == 0) {
          accn = tnl;
          acch = th;
        } else {
          accn = accn + tnl;
          acch = acch + th;
        }
      }
      anl[q][l] = accn;
      ah[q][l] = acch;
    }
  bool inside = good;
  for (int i = 0; i < m; i++) {
    double knl = 0.0, kh = 0.0;
    if (good) {
      double ynl = 0.0, yh = 0.0;
      for (int l = 0; l < m; l++) {
        double pnl, ph;
        point_times(Mm[((int64_t)i * m + l) * nleaf + b], -opaque(fc_lo[(int64_t)l * nleaf + b]),
                    fc_hi[(int64_t)l * nleaf + b], pnl, ph);
        if (l == 0) {
          ynl = pnl;
          yh = ph;
        } else {
          ynl = ynl + pnl;
          yh = yh + ph;
        }
      }
      knl = yh;  // -yf
      kh = ynl;
      for (int l = 0; l < m; l++) {
        double cnl = i == l ? -1.0 : opaque(-0.0), chh = i == l ? 1.0 : 0.0;
        for (int q = 0; q < m; q++) {
          double tnl, th;
          point_times(Mm[((int64_t)i * m + q) * nleaf + b], anl[q][l], ah[q][l], tnl, th);
          cnl = cnl + th;  // a - t
          chh = chh + tnl;
        }
        mul_add_sep(cnl, chh, Ycube, knl, kh);  // a Y + K_i
        knl = cnl;
        kh = chh;
      }
      inside = inside && (knl < r) && (kh < r);
    }
    if (kout) {
      kout[(b * m + i) * 2] = -opaque(knl);
      kout[(b * m + i) * 2 + 1] = kh;
    }
  }
  incl[b] = (uint8_t)inside;
}

struct NewtonPlan {
  double *fcl, *fch, *sl, *sh, *Y;
  uint8_t* ok;
  int32_t* labels;
  char* scratch;
  size_t scratch_bytes;
};

static size_t newton_scratch_bytes(const vx_poly* P, int np, const MvPolys& M, const vx_csf* S) {
  const int k = S->k;
  size_t e = eval_level_bytes(P, np, S);
  for (int j = 0; j < k; j++) {
    vx_poly col[VX_KMAX];
    for (int i = 0; i < k; i++) col[i] = M.dp[(size_t)i * k + j];
    const size_t ej = eval_level_bytes(col, k, S);
    e = ej > e ? ej : e;
  }
  return e;
}

static void plan_newton(Arena& A, NewtonPlan& N, const vx_poly* P, int np, const MvPolys& M, const vx_csf* S) {
  const int k = S->k;
  const size_t nl = (size_t)S->n[k - 1];
  N.fcl = A.take<double>(np * nl);
  N.fch = A.take<double>(np * nl);
  N.sl = A.take<double>((size_t)k * k * nl);
  N.sh = A.take<double>((size_t)k * k * nl);
  N.Y = A.take<double>((size_t)k * k * nl);
  N.ok = A.take<uint8_t>(nl);
  N.labels = A.take<int32_t>((size_t)k * nl);
  N.scratch_bytes = newton_scratch_bytes(P, np, M, S);
  N.scratch = A.take<char>(N.scratch_bytes);
}

struct SpanPlan {
  double *fcl, *fch, *gl, *gh, *dl, *dh, *G, *M;
  uint8_t* ok;
  int32_t* labels;
  char* scratch;
  size_t scratch_bytes;
};

static void plan_span(Arena& A, SpanPlan& N, const vx_poly* P, int np, const MvPolys& M, const vx_csf* S) {
  const int k = S->k;
  const size_t nl = (size_t)S->n[k - 1];
  N.fcl = A.take<double>(np * nl);
  N.fch = A.take<double>(np * nl);
  N.gl = A.take<double>((size_t)np * k * nl);
  N.gh = A.take<double>((size_t)np * k * nl);
  N.dl = A.take<double>((size_t)np * k * nl);
  N.dh = A.take<double>((size_t)np * k * nl);
  N.G = A.take<double>((size_t)k * np * nl);
  N.M = A.take<double>((size_t)np * np * nl);
  N.ok = A.take<uint8_t>(nl);
  N.labels = A.take<int32_t>((size_t)k * nl);
  N.scratch_bytes = mv_scratch_bytes(P, np, M, S);
  N.scratch = A.take<char>(N.scratch_bytes);
}

static GridSet grid_set(const double* dom, int k, int level) {
  GridSet gs;
  memset(&gs, 0, sizeof gs);
  for (int a = 0; a < k; a++) {
    AxisGrid g;
    g.dlo = dom[2 * a];
    g.dhi = dom[2 * a + 1];
    g.ndlo = -g.dlo;
    g.ndhi = -g.dhi;
    g.level = level;
    g.centre = 0;
    gs.cell[a] = g;
    g.centre = 1;
    gs.centre[a] = g;
    g.centre = 2;
    gs.vertex[a] = g;
  }
  return gs;
}

// The test for np < k polynomials (see k_span_m); K is np per box.
static int newton_span_impl(const vx_poly* P, int np, const vx_csf* S, const double* dom, uint8_t* incl,
                            double* kout, void* ws, size_t ws_bytes, hipStream_t st) {
  const int k = S->k;
  const int64_t nl = S->n[k - 1];
  if (nl == 0) return VX_OK;
  const size_t rb = (mv_run_bytes(P, np, 1) + 255) / 256 * 256;
  if (rb > ws_bytes) VX_FAIL(VX_ECAPACITY, "Newton test: workspace too small");
  MvRun R;
  int rc;
  if ((rc = mv_run_prepare(P, np, 1, reinterpret_cast<char*>(ws), rb, R, st))) return rc;
  Arena A;
  A.base = reinterpret_cast<char*>(ws) + rb;
  A.size = ws_bytes - rb;
  SpanPlan N;
  plan_span(A, N, P, np, R.M, S);
  if (A.overflow) VX_FAIL(VX_ECAPACITY, "Newton test: workspace of %zu bytes is too small", ws_bytes);
  const int pr = prof_start("newton", (double)nl, st);
  // F and its gradient at the centres, the gradient on the boxes
  if ((rc = eval_level_prepared(R.QF, S, dom, N.fcl, N.fch, nullptr, N.scratch, N.scratch_bytes, st, P, 1)))
    return rc;
  if ((rc = eval_level_prepared(R.QD, S, dom, N.gl, N.gh, nullptr, N.scratch, N.scratch_bytes, st, R.M.dp.data(),
                                1)))
    return rc;
  if ((rc = eval_level_prepared(R.QD, S, dom, N.dl, N.dh, nullptr, N.scratch, N.scratch_bytes, st, R.M.dp.data(),
                                0)))
    return rc;
  CsfView cv;
  memset(&cv, 0, sizeof cv);
  for (int l = 0; l < k; l++) {
    cv.idx[l] = S->idx[l];
    cv.ptr[l] = S->ptr[l];
    cv.n[l] = S->n[l];
  }
  const unsigned nb = (unsigned)((nl + 255) / 256);
  hipLaunchKernelGGL(k_leaf_labels, dim3(nb), dim3(256), 0, st, k, cv, N.labels);
  VX_CHECK_LAUNCH("k_leaf_labels");
  hipLaunchKernelGGL(k_span_m, dim3(nb), dim3(256), 0, st, k, np, nl, (const double*)N.gl, (const double*)N.gh,
                     (const double*)N.dl, (const double*)N.dh, N.G, N.M, N.ok);
  VX_CHECK_LAUNCH("k_span_m");
  hipLaunchKernelGGL(k_span_k, dim3(nb), dim3(256), 0, st, k, np, nl, grid_set(dom, k, S->level),
                     (const int32_t*)N.labels, (const double*)N.fcl, (const double*)N.fch, (const double*)N.dl,
                     (const double*)N.dh, (const double*)N.G, (const double*)N.M, (const uint8_t*)N.ok, incl, kout);
  VX_CHECK_LAUNCH("k_span_k");
  prof_stop(pr, st);
  return VX_OK;
}

size_t newton_workspace_bytes(const vx_poly* P, int np, const vx_csf* S) {
  MvPolys M = mv_polys(P, np, 1, nullptr, nullptr, nullptr, nullptr);
  if (np < S->k) {
    Arena A;
    SpanPlan N;
    plan_span(A, N, P, np, M, S);
    return (mv_run_bytes(P, np, 1) + 255) / 256 * 256 + A.off + 512;
  }
  Arena A;
  NewtonPlan N;
  plan_newton(A, N, P, np, M, S);
  return (mv_run_bytes(P, np, 1) + 255) / 256 * 256 + A.off + 512;
}

int newton_impl(const vx_poly* P, int np, const vx_csf* S, const double* dom, uint8_t* incl, double* kout, void* ws,
                size_t ws_bytes, hipStream_t st) {
  const int k = S->k;
  const int64_t nl = S->n[k - 1];
  if (np < k) return newton_span_impl(P, np, S, dom, incl, kout, ws, ws_bytes, st);
  if (nl == 0) return VX_OK;
  const size_t rb = (mv_run_bytes(P, np, 1) + 255) / 256 * 256;
  if (rb > ws_bytes) VX_FAIL(VX_ECAPACITY, "Newton test: workspace too small");
  MvRun R;
  int rc;
  if ((rc = mv_run_prepare(P, np, 1, reinterpret_cast<char*>(ws), rb, R, st))) return rc;
  Arena A;
  A.base = reinterpret_cast<char*>(ws) + rb;
  A.size = ws_bytes - rb;
  NewtonPlan N;
  plan_newton(A, N, P, np, R.M, S);
  if (A.overflow) VX_FAIL(VX_ECAPACITY, "Newton test: workspace of %zu bytes is too small", ws_bytes);
  const int pr = prof_start("newton", (double)nl, st);
  // F at the centres; slope column j: dF_i/dx_j with cells on axes 0..j and
  // centres on the others
  if ((rc = eval_level_prepared(R.QF, S, dom, N.fcl, N.fch, nullptr, N.scratch, N.scratch_bytes, st, P, 1)))
    return rc;
  for (int j = 0; j < k; j++) {
    int idx[VX_KMAX], modes[VX_KMAX];
    vx_poly col[VX_KMAX];
    for (int i = 0; i < k; i++) {
      idx[i] = i * k + j;
      col[i] = R.M.dp[(size_t)i * k + j];
    }
    for (int a = 0; a < k; a++) modes[a] = a <= j ? 0 : 1;
    const Prepared Qj = prepared_subset(R.QD, idx, k);
    if ((rc = eval_level_prepared(Qj, S, dom, N.sl + (size_t)j * k * nl, N.sh + (size_t)j * k * nl, nullptr,
                                  N.scratch, N.scratch_bytes, st, col, 0, modes)))
      return rc;
  }
  CsfView cv;
  memset(&cv, 0, sizeof cv);
  for (int l = 0; l < k; l++) {
    cv.idx[l] = S->idx[l];
    cv.ptr[l] = S->ptr[l];
    cv.n[l] = S->n[l];
  }
  const unsigned nb = (unsigned)((nl + 255) / 256);
  hipLaunchKernelGGL(k_leaf_labels, dim3(nb), dim3(256), 0, st, k, cv, N.labels);
  VX_CHECK_LAUNCH("k_leaf_labels");
  hipLaunchKernelGGL(k_newton_y, dim3(nb), dim3(256), 0, st, k, nl, (const double*)N.sl, (const double*)N.sh, N.Y,
                     N.ok);
  VX_CHECK_LAUNCH("k_newton_y");
  GridSet gs;
  memset(&gs, 0, sizeof gs);
  for (int a = 0; a < k; a++) {
    AxisGrid g;
    g.dlo = dom[2 * a];
    g.dhi = dom[2 * a + 1];
    g.ndlo = -g.dlo;
    g.ndhi = -g.dhi;
    g.level = S->level;
    g.centre = 0;
    gs.cell[a] = g;
    g.centre = 1;
    gs.centre[a] = g;
    g.centre = 2;
    gs.vertex[a] = g;
  }
  hipLaunchKernelGGL(k_newton_k, dim3(nb), dim3(256), 0, st, k, nl, gs, (const int32_t*)N.labels,
                     (const double*)N.fcl, (const double*)N.fch, (const double*)N.sl, (const double*)N.sh,
                     (const double*)N.Y, (const uint8_t*)N.ok, incl, kout);
  VX_CHECK_LAUNCH("k_newton_k");
  prof_stop(pr, st);
  return VX_OK;
}

// ---------------------------------------------------------------------------
// Variable order.  Theorem 1's cost sums, over the CSF depths, the trailing
// tuple counts times the node counts N_l(S), and the node counts depend on
// which axis each depth holds.  For an order pi (depth l holds axis pi[l])
// the node counts are those of the CSF built from the boxes' labels listed
// in that order.
// ---------------------------------------------------------------------------
struct AxisOrder {
  int a[VX_KMAX];
};

__global__ void k_order_labels(int k, int64_t n, AxisOrder o, const int32_t* __restrict__ in,
                               int32_t* __restrict__ out) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n) return;
  for (int l = 0; l < k; l++) out[b * k + l] = in[b * k + o.a[l]];
}

struct OrderPlan {
  int32_t* labels;
  int32_t* ordered;
  vx_csf T;
  size_t build_bytes;
  char* build_ws;
};

static void plan_order(Arena& A, OrderPlan& O, const vx_csf* S) {
  const int k = S->k;
  const int64_t n = S->n[k - 1] > 0 ? S->n[k - 1] : 1;
  O.labels = A.take<int32_t>((size_t)n * k);
  O.ordered = A.take<int32_t>((size_t)n * k);
  memset(&O.T, 0, sizeof O.T);
  O.T.k = k;
  O.T.level = S->level;
  for (int l = 0; l < k; l++) {
    O.T.cap[l] = n;
    O.T.idx[l] = A.take<int32_t>((size_t)n);
    if (l + 1 < k) O.T.ptr[l] = A.take<int32_t>((size_t)n + 1);
  }
  O.build_bytes = build_workspace_bytes(k, n);
  O.build_ws = A.take<char>(O.build_bytes);
}

size_t order_workspace_bytes(const vx_csf* S) {
  Arena A;
  OrderPlan O;
  plan_order(A, O, S);
  return A.off + 256;
}

int order_counts_impl(const vx_csf* S, int norders, const int32_t* orders, int64_t* counts, void* ws,
                      size_t ws_bytes, hipStream_t st) {
  const int k = S->k;
  const int64_t n = S->n[k - 1];
  if (n == 0) {
    for (int i = 0; i < norders * k; i++) counts[i] = 0;
    return VX_OK;
  }
  Arena A;
  A.base = reinterpret_cast<char*>(ws);
  A.size = ws_bytes;
  OrderPlan O;
  plan_order(A, O, S);
  if (A.overflow) VX_FAIL(VX_ECAPACITY, "variable_order_costs: workspace of %zu bytes is too small", ws_bytes);
  CsfView cv;
  memset(&cv, 0, sizeof cv);
  for (int l = 0; l < k; l++) {
    cv.idx[l] = S->idx[l];
    cv.ptr[l] = S->ptr[l];
    cv.n[l] = S->n[l];
  }
  const unsigned nb = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(k_leaf_labels, dim3(nb), dim3(256), 0, st, k, cv, O.labels);
  VX_CHECK_LAUNCH("k_leaf_labels");
  for (int o = 0; o < norders; o++) {
    AxisOrder ax;
    memset(&ax, 0, sizeof ax);
    for (int l = 0; l < k; l++) ax.a[l] = orders[o * k + l];
    hipLaunchKernelGGL(k_order_labels, dim3(nb), dim3(256), 0, st, k, n, ax, (const int32_t*)O.labels, O.ordered);
    VX_CHECK_LAUNCH("k_order_labels");
    int rc;
    if ((rc = build_impl(k, S->level, O.ordered, n, &O.T, nullptr, O.build_ws, O.build_bytes, st))) return rc;
    for (int l = 0; l < k; l++) counts[o * k + l] = O.T.n[l];
  }
  return VX_OK;
}

}  // namespace vx
