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
#include <hip/hip_runtime.h>
#include <string.h>

#include <vector>

#include "common.hpp"
#include "eval.hpp"
#include "interval.hpp"
#include "profile.hpp"

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
      step_gen(dnl, dh, W[i], anl, ah);  // D_i * W_i + acc
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

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------
struct MvPolys {
  std::vector<vx_poly> dp;  // derivative polynomials, (p, axis) order
  int64_t cube_max = 1;
};

static MvPolys mv_polys(const vx_poly* P, int np, double* dlo, double* dhi) {
  MvPolys M;
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
  return M;
}

static int launch_deriv(const vx_poly* P, int np, const MvPolys& M, double* dlo, double* dhi, hipStream_t st) {
  const int k = P[0].k;
  DerivArgs a;
  memset(&a, 0, sizeof a);
  for (int p = 0; p < np; p++) {
    a.clo[p] = P[p].c_lo;
    a.chi[p] = P[p].c_hi;
    a.d[p] = P[p].degree;
    a.side[p] = P[p].side;
  }
  hipLaunchKernelGGL(k_deriv, dim3((unsigned)((M.cube_max + 255) / 256), (unsigned)(np * k)), dim3(256), 0, st, a,
                     k, M.cube_max, dlo, dhi);
  VX_CHECK_LAUNCH("k_deriv");
  return VX_OK;
}

// Per-run state of the mean-value test: derivative coefficient cubes and the
// prepared tables of F and of its derivatives (built once).
struct MvRun {
  MvPolys M;
  Prepared QF, QD;
  double* dlo = nullptr;
  double* dhi = nullptr;
};

static size_t mv_run_bytes(const vx_poly* P, int np) {
  MvPolys M = mv_polys(P, np, nullptr, nullptr);
  const size_t cubes = ((sizeof(double) * (size_t)M.cube_max * np * P[0].k + 255) / 256 * 256) * 2;
  return cubes + prepared_bytes(P, np) + prepared_bytes(M.dp.data(), (int)M.dp.size()) + 1024;
}

static int mv_run_prepare(const vx_poly* P, int np, char* ws, size_t bytes, MvRun& R, hipStream_t st) {
  const int k = P[0].k;
  MvPolys M0 = mv_polys(P, np, nullptr, nullptr);
  const size_t cube_bytes = (sizeof(double) * (size_t)M0.cube_max * np * k + 255) / 256 * 256;
  R.dlo = reinterpret_cast<double*>(ws);
  R.dhi = reinterpret_cast<double*>(ws + cube_bytes);
  R.M = mv_polys(P, np, R.dlo, R.dhi);
  char* at = ws + 2 * cube_bytes;
  const size_t qf = (prepared_bytes(P, np) + 255) / 256 * 256;
  const size_t qd = (prepared_bytes(R.M.dp.data(), (int)R.M.dp.size()) + 255) / 256 * 256;
  if (2 * cube_bytes + qf + qd > bytes) VX_FAIL(VX_ECAPACITY, "mean-value test: workspace too small");
  int rc;
  if ((rc = launch_deriv(P, np, R.M, R.dlo, R.dhi, st))) return rc;
  if ((rc = prepare_polys(P, np, at, qf, &R.QF, st))) return rc;
  if ((rc = prepare_polys(R.M.dp.data(), (int)R.M.dp.size(), at + qf, qd, &R.QD, st))) return rc;
  return VX_OK;
}

static size_t mv_level_bytes(const vx_poly* P, int np, const MvPolys& M, const vx_csf* S) {
  const int k = S->k;
  const int64_t nl = S->n[k - 1];
  auto r = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t ef = eval_level_bytes(P, np, S), ed = eval_level_bytes(M.dp.data(), (int)M.dp.size(), S);
  return r(sizeof(double) * np * nl) * 2 + r(sizeof(double) * np * k * nl) * 2 + r(sizeof(int32_t) * k * nl) +
         (ef > ed ? ef : ed) + 256;
}

// One level: mean-value enclosures lo/hi (np x nleaf) and keep AND-ed.
static int mv_level(const vx_poly* P, int np, const MvRun& R, const vx_csf* S, const double* dom, double* lo,
                    double* hi, uint8_t* keep, char* ws, size_t bytes, hipStream_t st) {
  const int k = S->k;
  const int64_t nl = S->n[k - 1];
  if (nl == 0) return VX_OK;
  Arena A;
  A.base = ws;
  A.size = bytes;
  double* fcl = A.take<double>((size_t)np * nl);
  double* fch = A.take<double>((size_t)np * nl);
  double* dl = A.take<double>((size_t)np * k * nl);
  double* dh = A.take<double>((size_t)np * k * nl);
  int32_t* labels = A.take<int32_t>((size_t)k * nl);
  const size_t ef = eval_level_bytes(P, np, S), ed = eval_level_bytes(R.M.dp.data(), (int)R.M.dp.size(), S);
  char* scratch = A.take<char>(ef > ed ? ef : ed);
  if (A.overflow) VX_FAIL(VX_ECAPACITY, "mean-value test: workspace of %zu bytes is too small", bytes);
  const size_t sb = ef > ed ? ef : ed;
  const int pr = prof_start("mean_value", (double)nl, st);
  int rc;
  if ((rc = eval_level_prepared(R.QF, S, dom, fcl, fch, nullptr, scratch, sb, st, P, 1))) return rc;
  if ((rc = eval_level_prepared(R.QD, S, dom, dl, dh, nullptr, scratch, sb, st, R.M.dp.data(), 0))) return rc;
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
  }
  hipLaunchKernelGGL(k_mv_combine, dim3(nb), dim3(256), 0, st, k, np, nl, gs, (const int32_t*)labels,
                     (const double*)fcl, (const double*)fch, (const double*)dl, (const double*)dh, lo, hi, keep);
  VX_CHECK_LAUNCH("k_mv_combine");
  prof_stop(pr, st);
  return VX_OK;
}

size_t mv_workspace_bytes(const vx_poly* P, int np, const vx_csf* S) {
  MvPolys M = mv_polys(P, np, nullptr, nullptr);
  return mv_run_bytes(P, np) + mv_level_bytes(P, np, M, S) + 512;
}

int mv_impl(const vx_poly* P, int np, const vx_csf* S, const double* dom, double* lo, double* hi, uint8_t* keep,
            void* ws, size_t ws_bytes, hipStream_t st) {
  if (S->n[S->k - 1] == 0) return VX_OK;
  const size_t rb = (mv_run_bytes(P, np) + 255) / 256 * 256;
  if (rb > ws_bytes) VX_FAIL(VX_ECAPACITY, "mean_value_exclusion: workspace too small");
  MvRun R;
  int rc;
  if ((rc = mv_run_prepare(P, np, reinterpret_cast<char*>(ws), rb, R, st))) return rc;
  return mv_level(P, np, R, S, dom, lo, hi, keep, reinterpret_cast<char*>(ws) + rb, ws_bytes - rb, st);
}

// Run-level interface for run_subdivision: the tables are built once.
size_t mv_run_workspace(const vx_poly* P, int np) { return (mv_run_bytes(P, np) + 255) / 256 * 256; }

size_t mv_level_workspace(const vx_poly* P, int np, const vx_csf* S) {
  MvPolys M = mv_polys(P, np, nullptr, nullptr);
  return mv_level_bytes(P, np, M, S);
}

struct MvRunHandle {
  MvRun R;
};

void* mv_run_begin(const vx_poly* P, int np, void* ws, size_t bytes, hipStream_t st, int* rc) {
  MvRunHandle* h = new MvRunHandle;
  *rc = mv_run_prepare(P, np, reinterpret_cast<char*>(ws), bytes, h->R, st);
  if (*rc) {
    delete h;
    return nullptr;
  }
  return h;
}

int mv_run_level(void* handle, const vx_poly* P, int np, const vx_csf* S, const double* dom, double* lo, double* hi,
                 uint8_t* keep, void* ws, size_t bytes, hipStream_t st) {
  const MvRunHandle* h = reinterpret_cast<const MvRunHandle*>(handle);
  return mv_level(P, np, h->R, S, dom, lo, hi, keep, reinterpret_cast<char*>(ws), bytes, st);
}

void mv_run_end(void* handle) { delete reinterpret_cast<MvRunHandle*>(handle); }

}  // namespace vx
