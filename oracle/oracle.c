/*
 * oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow CPU reference for the interval-subdivision hot path of
 * G. Moroz, "Sparse Tensors and Subdivision Methods for Finding the Zero Set
 * of Polynomial Equations" (arXiv 2406.09857).  Only the tests, the smoke
 * check and the CPU-baseline leg of the benchmark load this library; the
 * product library never links, calls or includes anything from here, and this
 * file includes nothing from the product.
 *
 * What is computed (and where the paper defines it):
 *   - interval addition [a,b]+[c,d] = [a+c, b+d]  (Sec. 3.2, "Exclusion
 *     Criterion"), with every endpoint rounded outward (lower endpoints toward
 *     -inf, upper endpoints toward +inf) so that {F(x) : x in B} is contained
 *     in the result;
 *   - interval product [a,b]*[c,d] = [min P, max P], P = {ac, ad, bc, bd}, the
 *     textbook rule (the paper names interval arithmetic but does not spell the
 *     product out), with the min rounded down and the max rounded up;
 *   - Horner's rule on an interval (Algorithm 1): J <- a_l; J <- J*I + a_j for
 *     descending exponents (consecutive exponents, so I^(e_{j+1}-e_j) = I);
 *     each step J*I + a_j is taken as one interval operation: the exact range
 *     [min P + lo(a_j), max P + hi(a_j)] of that set, each endpoint rounded
 *     outward once (fma in the directed mode), the tightest floating-point
 *     enclosure of the step (the paper asks only for the enclosure property);
 *   - EvaluationCSF (Algorithm 2): for every x1 node i of the box CSF, the
 *     partial evaluation F(I_i, x2, ..., xk) and a recursive call on the
 *     subtree of i; a univariate F is evaluated directly on each child.
 *   - a per-box brute force that evaluates one box by nested Horner without
 *     sharing anything between boxes (the left-hand side of Theorem 1's
 *     comparison), used to pin the amortized routine;
 *   - the mean-value (order-1 Taylor form) enclosure of Sec. 3.2: centre
 *     enclosures, derivative coefficients and the final combination;
 *   - the Newton test for systems with fewer equations than variables
 *     (Sec. 3.2): the same test on the plane through the box spanned by the
 *     gradients at its centre;
 *   - the Newton interval inclusion test for square systems (Sec. 3.2) in
 *     Krawczyk's form, from slope enclosures;
 *   - the grid-vertex enclosures of the inclusion criterion C1 (Sec. 3.2) and
 *     its Taylor-based form (order-2 bounds at the two extreme vertices of
 *     the linear part);
 *   - the order-2 Taylor form of Sec. 3.2 (Taylor form definition, m = 2):
 *     second-derivative coefficients (halved on the diagonal) and the
 *     combination F(c) + sum_i dF/dx_i(c) W_i + sum_{i<=j} H_ij(B) W_i W_j,
 *     W_i = B_i - c_i, with the diagonal products taken as interval squares;
 *   - the Taylor form of any order m (the same definition): the coefficient
 *     polynomials D^alpha F / alpha! of every multi-index, the ranges of the
 *     powers (x_i - c_i)^a over the box, and the combination.
 *
 * Rounding is set with fesetround() around each batch of endpoint
 * computations; the file is compiled with clang -ffp-model=strict so that the
 * compiler neither folds nor reorders floating-point operations across the
 * mode changes (FENV_ACCESS ON below).
 *
 * Polynomials are dense coefficient cubes of side `cube` in k variables,
 * c[e1][e2]...[ek] in C order, restricted to the total-degree simplex
 * e1+...+ek <= d (entries outside are never read).  Coefficients are
 * intervals [clo, chi]; point coefficients pass the same array twice.
 */
#include <fenv.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#pragma STDC FENV_ACCESS ON

#define ORC_KMAX 4

/* Rounding modes of the oracle: OUTWARD is interval arithmetic proper;
 * NEAREST evaluates every endpoint in round-to-nearest (used to compare
 * degenerate boxes against an ordinary floating-point Horner evaluation). */
enum { ORC_OUTWARD = 0, ORC_NEAREST = 1 };

typedef struct { double lo, hi; } ivl;

static void round_down(int mode) { fesetround(mode == ORC_NEAREST ? FE_TONEAREST : FE_DOWNWARD); }
static void round_up(int mode) { fesetround(mode == ORC_NEAREST ? FE_TONEAREST : FE_UPWARD); }
static void round_restore(void) { fesetround(FE_TONEAREST); }

static double min4(double a, double b, double c, double d) { return fmin(fmin(a, b), fmin(c, d)); }
static double max4(double a, double b, double c, double d) { return fmax(fmax(a, b), fmax(c, d)); }

/* ------------------------------------------------------------------ */
/* Scalar interval operations (one rounding-mode switch per endpoint). */
/* ------------------------------------------------------------------ */

static ivl iv_add(ivl x, ivl y, int mode) {
  ivl r;
  round_down(mode); r.lo = x.lo + y.lo;
  round_up(mode);   r.hi = x.hi + y.hi;
  round_restore();
  return r;
}

static ivl iv_mul(ivl x, ivl y, int mode) {
  ivl r;
  round_down(mode); r.lo = min4(x.lo * y.lo, x.lo * y.hi, x.hi * y.lo, x.hi * y.hi);
  round_up(mode);   r.hi = max4(x.lo * y.lo, x.lo * y.hi, x.hi * y.lo, x.hi * y.hi);
  round_restore();
  return r;
}

/* The Horner step J*I + C of polynomial evaluation, as one interval
 * operation: the exact range [min P + c.lo, max P + c.hi] of the set
 * J*I + C (P = the four endpoint products), each endpoint rounded outward
 * once.  fma() rounds a*b + c once in the current mode, and RD/RU are
 * monotone, so RD(min P + c.lo) = min RD(p + c.lo) over p in P (and the same
 * for the max).  In NEAREST mode the step is the plain floating-point
 * J*I, then + C, as an ordinary Horner evaluation computes it. */
static ivl iv_muladd(ivl x, ivl y, ivl c, int mode) {
  if (mode == ORC_NEAREST) return iv_add(iv_mul(x, y, mode), c, mode);
  ivl r;
  round_down(mode);
  r.lo = min4(fma(x.lo, y.lo, c.lo), fma(x.lo, y.hi, c.lo), fma(x.hi, y.lo, c.lo), fma(x.hi, y.hi, c.lo));
  round_up(mode);
  r.hi = max4(fma(x.lo, y.lo, c.hi), fma(x.lo, y.hi, c.hi), fma(x.hi, y.lo, c.hi), fma(x.hi, y.hi, c.hi));
  round_restore();
  return r;
}

void orc_iv_add(const double* x, const double* y, int mode, double* r) {
  ivl a = {x[0], x[1]}, b = {y[0], y[1]};
  ivl s = iv_add(a, b, mode);
  r[0] = s.lo; r[1] = s.hi;
}

void orc_iv_mul(const double* x, const double* y, int mode, double* r) {
  ivl a = {x[0], x[1]}, b = {y[0], y[1]};
  ivl p = iv_mul(a, b, mode);
  r[0] = p.lo; r[1] = p.hi;
}

void orc_iv_muladd(const double* x, const double* y, const double* c, int mode, double* r) {
  ivl a = {x[0], x[1]}, b = {y[0], y[1]}, d = {c[0], c[1]};
  ivl p = iv_muladd(a, b, d, mode);
  r[0] = p.lo; r[1] = p.hi;
}

/* ------------------------------------------------------------------ */
/* Box intervals of the uniform grid G_n (Sec. 2.1, "Representing a Set */
/* of Boxes"), on a domain [dlo, dhi] split into n = 2^level cells.      */
/* Cell i is [dlo + i*w, dlo + (i+1)*w], w = (dhi-dlo)/2^level; its      */
/* enclosure rounds each endpoint outward.  On dyadic domains such as   */
/* [-1,1] every endpoint is exact.                                       */
/* ------------------------------------------------------------------ */

void orc_box(double dlo, double dhi, int level, int64_t label, double* r) {
  round_down(ORC_OUTWARD);
  double wd = dhi - dlo;
  double lo = dlo + ldexp((double)label * wd, -level);
  round_up(ORC_OUTWARD);
  double wu = dhi - dlo;
  double hi = dlo + ldexp((double)(label + 1) * wu, -level);
  round_restore();
  r[0] = lo; r[1] = hi;
}

void orc_box_table(double dlo, double dhi, int level, int64_t n, double* out) {
  for (int64_t i = 0; i < n; i++) orc_box(dlo, dhi, level, i, out + 2 * i);
}

/* ------------------------------------------------------------------ */
/* Tuple bookkeeping for dense cubes restricted to the simplex.         */
/* ------------------------------------------------------------------ */

static int64_t ipow(int64_t b, int e) { int64_t r = 1; while (e-- > 0) r *= b; return r; }

/* Total degree |t| of every flat index of an m-dimensional cube of side s. */
static int* degrees_of_cube(int m, int s) {
  int64_t n = ipow(s, m);
  int* deg = (int*)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
  for (int64_t f = 0; f < n; f++) {
    int64_t q = f; int g = 0;
    for (int j = 0; j < m; j++) { g += (int)(q % s); q /= s; }
    deg[f] = g;
  }
  return deg;
}

/* Flat indices of the m-dim cube with |t| <= d, listed by increasing |t|
 * (ties by flat index), and first[g] = number of tuples with |t| < g. */
typedef struct { int m, s, d; int64_t n; int64_t* flat; int64_t* first; int* deg; } graded;

static graded graded_make(int m, int s, int d) {
  graded G; G.m = m; G.s = s; G.d = d;
  int64_t cube = ipow(s, m);
  G.deg = degrees_of_cube(m, s);
  G.first = (int64_t*)calloc((size_t)d + 2, sizeof(int64_t));
  for (int64_t f = 0; f < cube; f++) if (G.deg[f] <= d) G.first[G.deg[f] + 1]++;
  for (int g = 0; g <= d; g++) G.first[g + 1] += G.first[g];
  G.n = G.first[d + 1];
  G.flat = (int64_t*)malloc(sizeof(int64_t) * (size_t)(G.n > 0 ? G.n : 1));
  int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * ((size_t)d + 1));
  for (int g = 0; g <= d; g++) fill[g] = G.first[g];
  for (int64_t f = 0; f < cube; f++) if (G.deg[f] <= d) G.flat[fill[G.deg[f]]++] = f;
  free(fill);
  return G;
}

static void graded_free(graded* G) { free(G->flat); free(G->first); free(G->deg); }

/* ------------------------------------------------------------------ */
/* Partial evaluation F(I, x_{s+1}, ..., x_k) of an m-variate interval  */
/* polynomial C (cube of side S over (e_s, t)) at the interval I: for    */
/* every trailing tuple t with |t| <= d, Horner in e_s from d-|t| down   */
/* to 0.  All chains sharing I advance together, one exponent at a time, */
/* so the rounding mode is switched twice per exponent, not per step.    */
/* Each chain performs exactly the steps of Algorithm 1, every step     */
/* J*I + c rounded outward once per endpoint (iv_muladd).               */
/* Out: cube of side S over t (m-1 dims), only |t| <= d written.         */
/* Returns the number of interval steps (one multiply-add each).         */
/* ------------------------------------------------------------------ */

static int64_t partial_eval(const ivl* C, int m, int S, int d, const graded* T, ivl I, int mode,
                            ivl* out, double* tmp) {
  int64_t tcube = ipow(S, m - 1), steps = 0;
  for (int e = d; e >= 0; e--) {
    /* chains with |t| < d-e continue, chains with |t| == d-e start at e. */
    int64_t nact = T->first[d - e];       /* tuples with |t| <= d-e-1 */
    int64_t nnew_end = T->first[d - e + 1];
    round_down(mode);
    for (int64_t j = 0; j < nact; j++) {
      int64_t f = T->flat[j];
      ivl J = out[f], c = C[(int64_t)e * tcube + f];
      tmp[j] = mode == ORC_NEAREST ? min4(J.lo * I.lo, J.lo * I.hi, J.hi * I.lo, J.hi * I.hi) + c.lo
                                   : min4(fma(J.lo, I.lo, c.lo), fma(J.lo, I.hi, c.lo), fma(J.hi, I.lo, c.lo),
                                          fma(J.hi, I.hi, c.lo));
    }
    round_up(mode);
    for (int64_t j = 0; j < nact; j++) {
      int64_t f = T->flat[j];
      ivl J = out[f], c = C[(int64_t)e * tcube + f];
      out[f].hi = mode == ORC_NEAREST ? max4(J.lo * I.lo, J.lo * I.hi, J.hi * I.lo, J.hi * I.hi) + c.hi
                                      : max4(fma(J.lo, I.lo, c.hi), fma(J.lo, I.hi, c.hi), fma(J.hi, I.lo, c.hi),
                                             fma(J.hi, I.hi, c.hi));
      out[f].lo = tmp[j];
    }
    round_restore();
    for (int64_t j = nact; j < nnew_end; j++) {
      int64_t f = T->flat[j];
      out[f] = C[(int64_t)e * tcube + f];
    }
    steps += nact;
  }
  return steps;
}

/* ------------------------------------------------------------------ */
/* Algorithm 2 (EvaluationCSF), recursive, on a box CSF.                 */
/* ------------------------------------------------------------------ */

typedef struct {
  int k, d, S, mode;
  const int64_t* n;           /* n[l] nodes at CSF depth l+1 */
  const int32_t* const* idx;  /* labels per depth */
  const int32_t* const* ptr;  /* child offsets per depth */
  const double* const* X;     /* X[l][2*label], X[l][2*label+1]: interval of that label on axis l */
  const int64_t* xn;          /* table sizes (labels must be < xn[l]) */
  graded T[ORC_KMAX];         /* T[l]: trailing tuples for stage l (dimension k-l-1) */
  double* lo; double* hi;     /* leaf outputs, CSF leaf order */
} csf_job;

typedef struct { ivl* buf[ORC_KMAX]; double* tmp; int64_t steps[ORC_KMAX]; int err; } csf_scratch;

/* Evaluate F (m = k - l variables, cube side S) on the nodes [b, e) of depth l. */
static void eval_rec(const csf_job* J, csf_scratch* W, const ivl* F, int l, int64_t b, int64_t e) {
  int m = J->k - l;
  for (int64_t q = b; q < e; q++) {
    int32_t lab = J->idx[l][q];
    if (lab < 0 || (int64_t)lab >= J->xn[l]) { W->err = 1; return; }
    ivl I = { J->X[l][2 * (int64_t)lab], J->X[l][2 * (int64_t)lab + 1] };
    ivl* FI = W->buf[l];
    W->steps[l] += partial_eval(F, m, J->S, J->d, &J->T[l], I, J->mode, FI, W->tmp);
    if (m == 1) {
      J->lo[q] = FI[0].lo; J->hi[q] = FI[0].hi;
    } else {
      eval_rec(J, W, FI, l + 1, J->ptr[l][q], J->ptr[l][q + 1]);
      if (W->err) return;
    }
  }
}

/*
 * Evaluate the polynomial (clo/chi: dense cube, side `cube`, degree d, k vars)
 * on every leaf of the box CSF (n, idx, ptr) whose axis-l labels index the
 * interval tables X[l] (2*xn[l] doubles).  Writes lo/hi in CSF leaf order and,
 * if steps != NULL, steps[l] = number of interval Horner steps spent at depth
 * l (for Theorem 1).  nthreads > 1 splits the x1 loop over OpenMP threads; the
 * result does not depend on it (every chain is sequential).
 * Returns 0, or -1 on bad arguments / out-of-table labels.
 */
int orc_eval_csf(int k, int d, int cube, const double* clo, const double* chi,
                 const int64_t* n, const int32_t* const* idx, const int32_t* const* ptr,
                 const double* const* X, const int64_t* xn, int mode, int nthreads,
                 double* lo, double* hi, int64_t* steps) {
  if (k < 1 || k > ORC_KMAX || d < 0 || cube < d + 1) return -1;
  csf_job J; memset(&J, 0, sizeof J);
  J.k = k; J.d = d; J.S = cube; J.mode = mode; J.n = n; J.idx = idx; J.ptr = ptr; J.X = X; J.xn = xn;
  J.lo = lo; J.hi = hi;
  for (int l = 0; l < k; l++) J.T[l] = graded_make(k - l - 1, cube, d);
  int64_t total = ipow(cube, k);
  ivl* F = (ivl*)malloc(sizeof(ivl) * (size_t)total);
  for (int64_t f = 0; f < total; f++) { F[f].lo = clo[f]; F[f].hi = chi ? chi[f] : clo[f]; }
  int64_t st[ORC_KMAX] = {0, 0, 0, 0};
  int err = 0;
  if (nthreads < 1) nthreads = 1;
#ifdef _OPENMP
#pragma omp parallel num_threads(nthreads) reduction(+ : err)
#endif
  {
    csf_scratch W; memset(&W, 0, sizeof W);
    for (int l = 0; l < k; l++) W.buf[l] = (ivl*)calloc((size_t)ipow(cube, k - l - 1), sizeof(ivl));
    W.tmp = (double*)malloc(sizeof(double) * (size_t)(J.T[0].n + 1));
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
    for (int64_t q = 0; q < n[0]; q++) {
      if (!W.err) eval_rec(&J, &W, F, 0, q, q + 1);
    }
#ifdef _OPENMP
#pragma omp critical
#endif
    { for (int l = 0; l < k; l++) st[l] += W.steps[l]; }
    err += W.err;
    for (int l = 0; l < k; l++) free(W.buf[l]);
    free(W.tmp);
  }
  round_restore();
  if (steps) for (int l = 0; l < k; l++) steps[l] = st[l];
  for (int l = 0; l < k; l++) graded_free(&J.T[l]);
  free(F);
  return err ? -1 : 0;
}

/* ------------------------------------------------------------------ */
/* Per-box brute force: nested Horner on one box, nothing shared.        */
/* value(s, rem, suffix) is the polynomial in x_1..x_s (suffix exponents */
/* e_{s+1..k} fixed, |e_1..e_s| <= rem) evaluated on I_1..I_s; the      */
/* outermost call is value(k, d, {}).  Every chain is Algorithm 1.      */
/* ------------------------------------------------------------------ */

typedef struct { int k, d, S, mode; const double* clo; const double* chi; const ivl* B; int64_t steps; } box_job;

static ivl box_value(box_job* J, int s, int rem, int* e) {
  /* e[0..k-1]: exponents; entries s..k-1 (0-based) are fixed by the caller. */
  ivl acc = {0.0, 0.0};
  for (int es = rem; es >= 0; es--) {
    e[s - 1] = es;
    ivl coef;
    if (s == 1) {
      int64_t f = 0;
      for (int j = 0; j < J->k; j++) f = f * J->S + e[j];
      coef.lo = J->clo[f]; coef.hi = J->chi ? J->chi[f] : J->clo[f];
    } else {
      coef = box_value(J, s - 1, rem - es, e);
    }
    if (es == rem) {
      acc = coef;
    } else {
      acc = iv_muladd(acc, J->B[s - 1], coef, J->mode);
      J->steps++;
    }
  }
  return acc;
}

/* Evaluate one box B (2k doubles: lo_1, hi_1, ..., lo_k, hi_k). */
int orc_eval_box(int k, int d, int cube, const double* clo, const double* chi, const double* box,
                 int mode, double* r, int64_t* steps) {
  if (k < 1 || k > ORC_KMAX || d < 0 || cube < d + 1) return -1;
  ivl B[ORC_KMAX];
  for (int j = 0; j < k; j++) { B[j].lo = box[2 * j]; B[j].hi = box[2 * j + 1]; }
  box_job J = {k, d, cube, mode, clo, chi, B, 0};
  int e[ORC_KMAX] = {0, 0, 0, 0};
  ivl v = box_value(&J, k, d, e);
  r[0] = v.lo; r[1] = v.hi;
  if (steps) *steps = J.steps;
  return 0;
}

/* Point evaluation in round-to-nearest by the same nested Horner order
 * (degenerate boxes); used by the derivative checks. */
int orc_eval_points(int k, int d, int cube, const double* c, const double* x, int64_t npts, double* f) {
  if (k < 1 || k > ORC_KMAX) return -1;
  for (int64_t p = 0; p < npts; p++) {
    double box[2 * ORC_KMAX], r[2];
    for (int j = 0; j < k; j++) { box[2 * j] = x[p * k + j]; box[2 * j + 1] = x[p * k + j]; }
    if (orc_eval_box(k, d, cube, c, NULL, box, ORC_NEAREST, r, NULL)) return -1;
    f[p] = r[0];
  }
  return 0;
}

/* ------------------------------------------------------------------ */
/* Mean-value exclusion: the Taylor form of order 1 (Sec. 3.2, Taylor    */
/* form definition with m = 1):  T(F, B) = F(c) + sum_i dF/dx_i(B) *     */
/* (B_i - c_i), c the centre of B.  Every part is an outward-rounded     */
/* enclosure: F(c) is the interval evaluation at the degenerate box of   */
/* the centre enclosures, dF/dx_i(B) the interval evaluation of the      */
/* derivative polynomial on B, B_i - c_i = [RD(lo_i - chi_i),            */
/* RU(hi_i - clo_i)], and the sum runs left to right over i.             */
/* ------------------------------------------------------------------ */

/* Enclosure of the centre of cell `label` at `level`: it is the common
 * endpoint of cells 2*label and 2*label+1 at level+1, so its lower bound is
 * the lower end of cell 2*label+1 and its upper bound the upper end of cell
 * 2*label (both exact on dyadic domains). */
void orc_centre(double dlo, double dhi, int level, int64_t label, double* r) {
  double a[2], b[2];
  orc_box(dlo, dhi, level + 1, 2 * label + 1, a);
  orc_box(dlo, dhi, level + 1, 2 * label, b);
  r[0] = a[0]; r[1] = b[1];
}

void orc_centre_table(double dlo, double dhi, int level, int64_t n, double* out) {
  for (int64_t i = 0; i < n; i++) orc_centre(dlo, dhi, level, i, out + 2 * i);
}

/* Enclosure of grid vertex v (0 <= v <= 2^level), the common endpoint of
 * cells v - 1 and v: the lower end of cell v and the upper end of cell v - 1
 * (exact on dyadic domains). */
void orc_vertex(double dlo, double dhi, int level, int64_t v, double* r) {
  double a[2], b[2];
  orc_box(dlo, dhi, level, v, a);
  orc_box(dlo, dhi, level, v - 1, b);
  r[0] = a[0]; r[1] = b[1];
}

void orc_vertex_table(double dlo, double dhi, int level, int64_t n, double* out) {
  for (int64_t i = 0; i < n; i++) orc_vertex(dlo, dhi, level, i, out + 2 * i);
}

/* Coefficients of dF/dx_axis: entry e is (e_axis + 1) * c_{e + u_axis},
 * rounded outward (the factor is positive, so the bounds scale separately).
 * Output cube of the same side; entries with |e| > d - 1 are zero. */
int orc_deriv(int k, int d, int cube, const double* clo, const double* chi, int axis, double* olo, double* ohi) {
  if (k < 1 || k > ORC_KMAX || axis < 0 || axis >= k || cube < d + 1) return -1;
  int64_t total = ipow(cube, k), stride = ipow(cube, k - 1 - axis);
  for (int64_t f = 0; f < total; f++) {
    int64_t q = f; int deg = 0, ea = 0;
    for (int j = k - 1; j >= 0; j--) {
      int e = (int)(q % cube); q /= cube;
      deg += e;
      if (j == axis) ea = e;
    }
    olo[f] = 0.0; ohi[f] = 0.0;
    if (deg + 1 > d || ea + 1 >= cube) continue;
    double n = (double)(ea + 1);
    int64_t src = f + stride;
    round_down(ORC_OUTWARD); olo[f] = n * clo[src];
    round_up(ORC_OUTWARD);   ohi[f] = n * (chi ? chi[src] : clo[src]);
    round_restore();
  }
  return 0;
}

/* Combine per box b: fc[b] (2), D[i][b] (2, axis i), box[b][i] and
 * centre[b][i] (2 each); out[b] = fc + D_0 W_0 + ... + D_{k-1} W_{k-1}. */
int orc_mean_value(int k, int64_t nbox, const double* fc, const double* D, const double* box,
                   const double* centre, double* out) {
  if (k < 1 || k > ORC_KMAX) return -1;
  for (int64_t b = 0; b < nbox; b++) {
    ivl acc = {fc[2 * b], fc[2 * b + 1]};
    for (int i = 0; i < k; i++) {
      const double* I = box + (b * k + i) * 2;
      const double* c = centre + (b * k + i) * 2;
      ivl W;
      round_down(ORC_OUTWARD); W.lo = I[0] - c[1];
      round_up(ORC_OUTWARD);   W.hi = I[1] - c[0];
      round_restore();
      ivl Di = {D[((int64_t)i * nbox + b) * 2], D[((int64_t)i * nbox + b) * 2 + 1]};
      acc = iv_add(acc, iv_mul(Di, W, ORC_OUTWARD), ORC_OUTWARD);
    }
    out[2 * b] = acc.lo; out[2 * b + 1] = acc.hi;
  }
  return 0;
}

/* Coefficients of H_ij, the order-2 Taylor coefficient polynomial of the
 * pair i <= j: (1/2) d2F/dx_i^2 for i == j, d2F/dx_i dx_j for i < j.  Entry e
 * is m * c_{e + u_i + u_j} with the integer m = (e_i+1)(e_i+2)/2 (i == j) or
 * (e_i+1)(e_j+1) (i < j), exact in double, times the coefficient rounded
 * outward once (m > 0, so the bounds scale separately).  Output cube of the
 * same side; entries with |e| > d - 2 are zero. */
int orc_deriv2(int k, int d, int cube, const double* clo, const double* chi, int i, int j, double* olo,
               double* ohi) {
  if (k < 1 || k > ORC_KMAX || i < 0 || j < i || j >= k || cube < d + 1) return -1;
  int64_t total = ipow(cube, k);
  int64_t shift = ipow(cube, k - 1 - i) + ipow(cube, k - 1 - j);
  for (int64_t f = 0; f < total; f++) {
    int64_t q = f; int deg = 0, ei = 0, ej = 0;
    for (int a = k - 1; a >= 0; a--) {
      int e = (int)(q % cube); q /= cube;
      deg += e;
      if (a == i) ei = e;
      if (a == j) ej = e;
    }
    olo[f] = 0.0; ohi[f] = 0.0;
    if (deg + 2 > d) continue;
    double m = i == j ? (double)((ei + 1) * (ei + 2) / 2) : (double)((ei + 1) * (ej + 1));
    int64_t src = f + shift;
    round_down(ORC_OUTWARD); olo[f] = m * clo[src];
    round_up(ORC_OUTWARD);   ohi[f] = m * (chi ? chi[src] : clo[src]);
    round_restore();
  }
  return 0;
}

/* Interval square: the range of x^2 over X (not X*X, which forgets that both
 * factors are the same variable). */
static ivl iv_sqr(ivl x) {
  ivl r;
  if (x.lo >= 0.0) {
    round_down(ORC_OUTWARD); r.lo = x.lo * x.lo;
    round_up(ORC_OUTWARD);   r.hi = x.hi * x.hi;
  } else if (x.hi <= 0.0) {
    round_down(ORC_OUTWARD); r.lo = x.hi * x.hi;
    round_up(ORC_OUTWARD);   r.hi = x.lo * x.lo;
  } else {
    r.lo = 0.0;
    round_up(ORC_OUTWARD); r.hi = fmax(x.lo * x.lo, x.hi * x.hi);
  }
  round_restore();
  return r;
}

/* Order-2 Taylor form per box b: fc[b] (2) = F(c), Dc[i][b] (2) = dF/dx_i(c),
 * H[t][b] (2) = H_ij(B) for the pairs t = (i, j), i <= j, in lexicographic
 * order, box[b][i] and centre[b][i] (2 each).  With W_i = B_i - c_i,
 *   out[b] = fc + Dc_0 W_0 + ... + Dc_{k-1} W_{k-1} + sum_t H_t X_t,
 * X_t = W_i^2 (i == j) or W_i W_j, summed left to right in that order. */
int orc_taylor2(int k, int64_t nbox, const double* fc, const double* Dc, const double* H, const double* box,
                const double* centre, double* out) {
  if (k < 1 || k > ORC_KMAX) return -1;
  for (int64_t b = 0; b < nbox; b++) {
    ivl W[ORC_KMAX];
    for (int i = 0; i < k; i++) {
      const double* I = box + (b * k + i) * 2;
      const double* c = centre + (b * k + i) * 2;
      round_down(ORC_OUTWARD); W[i].lo = I[0] - c[1];
      round_up(ORC_OUTWARD);   W[i].hi = I[1] - c[0];
      round_restore();
    }
    ivl acc = {fc[2 * b], fc[2 * b + 1]};
    for (int i = 0; i < k; i++) {
      ivl Di = {Dc[((int64_t)i * nbox + b) * 2], Dc[((int64_t)i * nbox + b) * 2 + 1]};
      acc = iv_add(acc, iv_mul(Di, W[i], ORC_OUTWARD), ORC_OUTWARD);
    }
    int t = 0;
    for (int i = 0; i < k; i++)
      for (int j = i; j < k; j++, t++) {
        ivl X = i == j ? iv_sqr(W[i]) : iv_mul(W[i], W[j], ORC_OUTWARD);
        ivl Ht = {H[((int64_t)t * nbox + b) * 2], H[((int64_t)t * nbox + b) * 2 + 1]};
        acc = iv_add(acc, iv_mul(Ht, X, ORC_OUTWARD), ORC_OUTWARD);
      }
    out[2 * b] = acc.lo; out[2 * b + 1] = acc.hi;
  }
  return 0;
}

/* ------------------------------------------------------------------ */
/* Taylor form of general order m (Sec. 3.2, Taylor form definition).  */
/* ------------------------------------------------------------------ */

/* In k variables the term of order j of the Taylor expansion at c is
 * sum_{|alpha| = j} (D^alpha F / alpha!) (x - c)^alpha (the multinomial form
 * of F^(j)(c) (x - c)^j / j!).  The coefficient polynomial D^alpha F / alpha!
 * has entry e = prod_i C(e_i + alpha_i, alpha_i) * c_{e + alpha}: an exact
 * integer times the coefficient, rounded outward once.  The integer must stay
 * below 2^53 (exact in double); -2 otherwise.  Output cube of the same side;
 * entries with |e| > d - |alpha| are zero.  |alpha| = 1 gives orc_deriv's
 * coefficients, |alpha| = 2 orc_deriv2's. */
static int64_t binom_exact(int n, int r) {
  int64_t v = 1;
  for (int i = 1; i <= r; i++) v = v * (n - r + i) / i;
  return v;
}

int orc_taylor_coef(int k, int d, int cube, const double* clo, const double* chi, const int* alpha, double* olo,
                    double* ohi) {
  if (k < 1 || k > ORC_KMAX || cube < d + 1) return -1;
  int order = 0;
  int64_t shift = 0;
  for (int i = 0; i < k; i++) {
    if (alpha[i] < 0) return -1;
    order += alpha[i];
    shift += alpha[i] * ipow(cube, k - 1 - i);
  }
  int64_t total = ipow(cube, k);
  for (int64_t f = 0; f < total; f++) {
    int64_t q = f; int deg = 0; int e[ORC_KMAX];
    for (int a = k - 1; a >= 0; a--) { e[a] = (int)(q % cube); q /= cube; deg += e[a]; }
    olo[f] = 0.0; ohi[f] = 0.0;
    if (deg + order > d) continue;
    /* prod_i C(e_i + alpha_i, alpha_i), checked against 2^53 */
    double m = 1.0;
    for (int i = 0; i < k; i++) {
      const int64_t b = binom_exact(e[i] + alpha[i], alpha[i]);
      m *= (double)b;
      if (m >= 9007199254740992.0) return -2;
    }
    int64_t src = f + shift;
    round_down(ORC_OUTWARD); olo[f] = m * clo[src];
    round_up(ORC_OUTWARD);   ohi[f] = m * (chi ? chi[src] : clo[src]);
    round_restore();
  }
  return 0;
}

/* Range of x^a over X (a >= 0), rounded outward: the power of one variable,
 * not the product X*X*...*X.  Powers of nonnegative values are formed left
 * to right by repeated multiplication (p <- p*v) in the direction of the
 * bound; odd powers are increasing, even powers have their minimum at the
 * point of X closest to 0. */
static double pow_up(double v, int a) { /* RU(v^a), v >= 0 */
  round_up(ORC_OUTWARD);
  double p = v;
  for (int i = 1; i < a; i++) p = p * v;
  round_restore();
  return p;
}
static double pow_down(double v, int a) { /* RD(v^a), v >= 0 */
  round_down(ORC_OUTWARD);
  double p = v;
  for (int i = 1; i < a; i++) p = p * v;
  round_restore();
  return p;
}

static ivl iv_pow(ivl x, int a) {
  ivl r;
  if (a == 0) { r.lo = 1.0; r.hi = 1.0; return r; }
  if (a == 1) return x;
  if (a % 2 == 1) {
    r.lo = x.lo >= 0.0 ? pow_down(x.lo, a) : -pow_up(-x.lo, a);
    r.hi = x.hi >= 0.0 ? pow_up(x.hi, a) : -pow_down(-x.hi, a);
  } else if (x.lo >= 0.0) {
    r.lo = pow_down(x.lo, a); r.hi = pow_up(x.hi, a);
  } else if (x.hi <= 0.0) {
    r.lo = pow_down(-x.hi, a); r.hi = pow_up(-x.lo, a);
  } else {
    r.lo = 0.0; r.hi = pow_up(fmax(-x.lo, x.hi), a);
  }
  return r;
}

/* The order-m Taylor form per box b from the enclosures of its terms:
 * terms[t][b] (2) for t = 0..nt-1, the multi-indices alpha[t] (k each) in the
 * order of the sum: |alpha| = 0 (F(c)) first, then orders 1..m, each order's
 * multi-indices as the non-decreasing index tuples i_1 <= ... <= i_j in
 * lexicographic order.  With W_i = B_i - c_i = [RD(lo_i - chi_i),
 * RU(hi_i - clo_i)] from box[b][i] and centre[b][i] (2 each),
 *   out[b] = terms_0 + sum_{t >= 1} terms_t X_t,
 *   X_t = prod_i W_i^alpha_i (ranges of powers, multiplied over ascending i),
 * summed left to right.  The caller evaluates the terms of orders below m
 * at the centre and those of order m over the box. */
int orc_taylor_m(int k, int nt, const int* alpha, int64_t nbox, const double* terms, const double* box,
                 const double* centre, double* out) {
  if (k < 1 || k > ORC_KMAX || nt < 1) return -1;
  for (int64_t b = 0; b < nbox; b++) {
    ivl W[ORC_KMAX];
    for (int i = 0; i < k; i++) {
      const double* I = box + (b * k + i) * 2;
      const double* c = centre + (b * k + i) * 2;
      round_down(ORC_OUTWARD); W[i].lo = I[0] - c[1];
      round_up(ORC_OUTWARD);   W[i].hi = I[1] - c[0];
      round_restore();
    }
    ivl acc = {terms[2 * b], terms[2 * b + 1]};
    for (int t = 1; t < nt; t++) {
      ivl X = {1.0, 1.0};
      int first = 1;
      for (int i = 0; i < k; i++) {
        const int a = alpha[t * k + i];
        if (a == 0) continue;
        const ivl P = iv_pow(W[i], a);
        X = first ? P : iv_mul(X, P, ORC_OUTWARD);
        first = 0;
      }
      ivl T = {terms[((int64_t)t * nbox + b) * 2], terms[((int64_t)t * nbox + b) * 2 + 1]};
      acc = iv_add(acc, iv_mul(T, X, ORC_OUTWARD), ORC_OUTWARD);
    }
    out[2 * b] = acc.lo; out[2 * b + 1] = acc.hi;
  }
  return 0;
}

/* Taylor-based inclusion criterion (Sec. 3.2, inclusion criterion from a
 * Taylor form of order m >= 2, here m = 2).  Per box: the linear part
 * l(x) = F(c) + grad F(c).(x - c) is largest at the vertex V_max that takes,
 * on axis i, the upper end when the enclosure of dF/dx_i(c) has lo + hi >= 0
 * (its midpoint is >= 0) and the lower end otherwise, and smallest at the
 * opposite vertex V_min.  F at a vertex V is bounded by the order-2 form at
 * the point V: F(c) + sum_i Dc_i (V_i - c_i) + sum_t H_t(B) X_t(V), with
 * V_i - c_i = [RD(vlo_i - chi_i), RU(vhi_i - clo_i)] from V's enclosure and
 * X_t the squares and products of those.  out[b] = 1 when the lower bound at
 * V_max is > 0 and the upper bound at V_min is < 0.  vlo_/vhi_ hold the
 * enclosures of each box's lower and upper vertex on every axis. */
static ivl taylor2_at(int k, int64_t nbox, int64_t b, ivl fc, const double* Dc, const double* H, const ivl* W) {
  ivl acc = fc;
  for (int i = 0; i < k; i++) {
    ivl Di = {Dc[((int64_t)i * nbox + b) * 2], Dc[((int64_t)i * nbox + b) * 2 + 1]};
    acc = iv_add(acc, iv_mul(Di, W[i], ORC_OUTWARD), ORC_OUTWARD);
  }
  int t = 0;
  for (int i = 0; i < k; i++)
    for (int j = i; j < k; j++, t++) {
      ivl X = i == j ? iv_sqr(W[i]) : iv_mul(W[i], W[j], ORC_OUTWARD);
      ivl Ht = {H[((int64_t)t * nbox + b) * 2], H[((int64_t)t * nbox + b) * 2 + 1]};
      acc = iv_add(acc, iv_mul(Ht, X, ORC_OUTWARD), ORC_OUTWARD);
    }
  return acc;
}

int orc_taylor_inclusion(int k, int64_t nbox, const double* fc, const double* Dc, const double* H,
                         const double* vlo_, const double* vhi_, const double* centre, uint8_t* out) {
  if (k < 1 || k > ORC_KMAX) return -1;
  for (int64_t b = 0; b < nbox; b++) {
    ivl Wmax[ORC_KMAX], Wmin[ORC_KMAX];
    for (int i = 0; i < k; i++) {
      const double* lv = vlo_ + (b * k + i) * 2;  /* lower vertex on axis i */
      const double* uv = vhi_ + (b * k + i) * 2;  /* upper vertex on axis i */
      const double* c = centre + (b * k + i) * 2;
      const double dlo = Dc[((int64_t)i * nbox + b) * 2], dhi = Dc[((int64_t)i * nbox + b) * 2 + 1];
      const int up = -dlo <= dhi;  /* lo + hi >= 0, exactly */
      const double* vmax = up ? uv : lv;
      const double* vmin = up ? lv : uv;
      round_down(ORC_OUTWARD); Wmax[i].lo = vmax[0] - c[1]; Wmin[i].lo = vmin[0] - c[1];
      round_up(ORC_OUTWARD);   Wmax[i].hi = vmax[1] - c[0]; Wmin[i].hi = vmin[1] - c[0];
      round_restore();
    }
    ivl f = {fc[2 * b], fc[2 * b + 1]};
    ivl tmax = taylor2_at(k, nbox, b, f, Dc, H, Wmax);
    ivl tmin = taylor2_at(k, nbox, b, f, Dc, H, Wmin);
    out[b] = (tmax.lo > 0.0 && tmin.hi < 0.0) ? 1 : 0;
  }
  return 0;
}

/* Newton interval inclusion test for a square system F = (F_1..F_k)
 * (Sec. 3.2, inclusion criterion for several polynomials), in Krawczyk's
 * form: with S the slope matrix of the box (S_ij enclosed by dF_i/dx_j on
 * the box with the first j variables free and the rest at the centre) and
 * Y = (mid S)^-1,
 *   K(B) = c - Y F(c) + (I - Y S)(B - c);
 * K(B) inside B gives a point where Y F = 0, hence F = 0 (Brouwer).  Per box:
 *   fc[i][b] (2)      F_i(c) enclosure,
 *   Sm[(i*k+j)][b] (2) S_ij enclosure,
 *   box, centre       outer box and centre enclosures (b, axis, 2),
 *   inner             inner box (b, axis, 2): [upper end of the lower vertex
 *                     enclosure, lower end of the upper vertex enclosure],
 *                     inside the true box;
 * Y in round-to-nearest: mid = (lo + hi) * 0.5, Gauss-Jordan with partial
 * pivoting (first largest |pivot|, rows swapped in A and Y, the pivot row
 * divided by the pivot, then r -= f * pivot row for r != col, columns in
 * ascending order); a zero pivot means no certificate.  K in outward
 * arithmetic: Yf_i = sum_j Y_ij F_j(c) (j ascending), A_ij = delta_ij -
 * sum_l Y_il S_lj (l ascending), K_i = (c_i - Yf_i) + sum_j A_ij W_j
 * (j ascending), W_j = B_j - c_j.  out[b] = 1 when every K_i lies in the
 * inner box; K (b, axis, 2) is written when not NULL. */
int orc_krawczyk(int k, int64_t nbox, const double* fc, const double* Sm, const double* box, const double* centre,
                 const double* inner, uint8_t* out, double* K) {
  if (k < 1 || k > ORC_KMAX) return -1;
  for (int64_t b = 0; b < nbox; b++) {
    double A[ORC_KMAX][ORC_KMAX], Y[ORC_KMAX][ORC_KMAX];
    round_restore();
    for (int i = 0; i < k; i++)
      for (int j = 0; j < k; j++) {
        const double* e = Sm + (((int64_t)(i * k + j)) * nbox + b) * 2;
        A[i][j] = (e[0] + e[1]) * 0.5;
        Y[i][j] = i == j ? 1.0 : 0.0;
      }
    int ok = 1;
    for (int col = 0; col < k && ok; col++) {
      int piv = col;
      for (int r = col + 1; r < k; r++)
        if (fabs(A[r][col]) > fabs(A[piv][col])) piv = r;
      if (!(A[piv][col] != 0.0)) { ok = 0; break; }  /* zero (or NaN) pivot */
      if (piv != col)
        for (int j = 0; j < k; j++) {
          double t = A[col][j]; A[col][j] = A[piv][j]; A[piv][j] = t;
          t = Y[col][j]; Y[col][j] = Y[piv][j]; Y[piv][j] = t;
        }
      const double p = A[col][col];
      for (int j = 0; j < k; j++) { A[col][j] = A[col][j] / p; Y[col][j] = Y[col][j] / p; }
      for (int r = 0; r < k; r++) {
        if (r == col) continue;
        const double f = A[r][col];
        for (int j = 0; j < k; j++) {
          A[r][j] = A[r][j] - f * A[col][j];
          Y[r][j] = Y[r][j] - f * Y[col][j];
        }
      }
    }
    int inside = ok;
    for (int i = 0; i < k; i++) {
      ivl Ki = {0.0, 0.0};
      if (ok) {
        ivl yf = {0.0, 0.0};
        for (int j = 0; j < k; j++) {
          ivl fj = {fc[((int64_t)j * nbox + b) * 2], fc[((int64_t)j * nbox + b) * 2 + 1]};
          ivl yj = {Y[i][j], Y[i][j]};
          yf = j == 0 ? iv_mul(yj, fj, ORC_OUTWARD) : iv_add(yf, iv_mul(yj, fj, ORC_OUTWARD), ORC_OUTWARD);
        }
        const double* c = centre + (b * k + i) * 2;
        ivl ci = {c[0], c[1]};
        ivl nyf = {-yf.hi, -yf.lo};
        Ki = iv_add(ci, nyf, ORC_OUTWARD);
        for (int j = 0; j < k; j++) {
          ivl a = {i == j ? 1.0 : 0.0, i == j ? 1.0 : 0.0};
          for (int l = 0; l < k; l++) {
            const double* e = Sm + (((int64_t)(l * k + j)) * nbox + b) * 2;
            ivl sl = {e[0], e[1]};
            ivl yl = {Y[i][l], Y[i][l]};
            ivl t = iv_mul(yl, sl, ORC_OUTWARD);
            ivl nt = {-t.hi, -t.lo};
            a = iv_add(a, nt, ORC_OUTWARD);
          }
          const double* I = box + (b * k + j) * 2;
          const double* cj = centre + (b * k + j) * 2;
          ivl W;
          round_down(ORC_OUTWARD); W.lo = I[0] - cj[1];
          round_up(ORC_OUTWARD);   W.hi = I[1] - cj[0];
          round_restore();
          Ki = iv_add(Ki, iv_mul(a, W, ORC_OUTWARD), ORC_OUTWARD);
        }
        const double* in = inner + (b * k + i) * 2;
        if (!(Ki.lo >= in[0] && Ki.hi <= in[1])) inside = 0;
      }
      if (K) { K[(b * k + i) * 2] = Ki.lo; K[(b * k + i) * 2 + 1] = Ki.hi; }
    }
    out[b] = (uint8_t)inside;
  }
  return 0;
}

/* Newton test for fewer equations than variables (Sec. 3.2, inclusion
 * criterion, last paragraph: intersect the box with the span of the
 * gradients at its centre, then apply the Newton test to the resulting
 * square system).  m < k polynomials.  Per box: the point c (the lower end
 * of the centre enclosure on every axis), G (k x m, column l = the midpoint
 * of F_l's gradient enclosure at the centre), the square system
 * phi(y) = F(c + G y) on the cube Y = [-r, r]^m, r the largest power of two
 * with c + G Y inside the box, and Krawczyk's operator
 *   K(Y) = -M phi(0) + (I - M A) Y,   A = D G (D: the Jacobian enclosed on
 *   the box, so A encloses phi's Jacobian on Y),   M = (mid(D) G)^-1.
 * K inside the open cube certifies a zero of phi in Y, that is a zero of F
 * in c + G Y, inside the box.
 *   fc   : m x nbox x 2, F_i on the centre enclosures (contains F_i(c));
 *   gc   : (m k) x nbox x 2, dF_i/dx_j on the centre enclosures, row i k + j;
 *   D    : (m k) x nbox x 2, dF_i/dx_j on the boxes;
 *   box, centre : nbox x k x 2.
 * G, mid(D) G and M are computed in round-to-nearest (any real M is valid);
 * every enclosure is outward.  out[b] = 1 when certified; K (nbox x m x 2)
 * and r (nbox) when not NULL (0 when no cube was found). */
int orc_newton_span(int k, int m, int64_t nbox, const double* fc, const double* gc, const double* D,
                    const double* box, const double* centre, uint8_t* out, double* K, double* rout) {
  if (k < 2 || k > ORC_KMAX || m < 1 || m >= k) return -1;
  for (int64_t b = 0; b < nbox; b++) {
    double G[ORC_KMAX][ORC_KMAX], P[ORC_KMAX][ORC_KMAX], Mi[ORC_KMAX][ORC_KMAX];
    round_restore();
    for (int j = 0; j < k; j++)
      for (int l = 0; l < m; l++) {
        const double* e = gc + (((int64_t)(l * k + j)) * nbox + b) * 2;
        G[j][l] = (e[0] + e[1]) * 0.5;
      }
    for (int i = 0; i < m; i++)
      for (int l = 0; l < m; l++) {
        double acc = 0.0;
        for (int j = 0; j < k; j++) {
          const double* e = D + (((int64_t)(i * k + j)) * nbox + b) * 2;
          const double t = ((e[0] + e[1]) * 0.5) * G[j][l];
          acc = j == 0 ? t : acc + t;
        }
        P[i][l] = acc;
        Mi[i][l] = i == l ? 1.0 : 0.0;
      }
    int ok = 1;
    for (int col = 0; col < m && ok; col++) {
      int piv = col;
      for (int r = col + 1; r < m; r++)
        if (fabs(P[r][col]) > fabs(P[piv][col])) piv = r;
      if (!(P[piv][col] != 0.0)) { ok = 0; break; }  /* zero (or NaN) pivot */
      if (piv != col)
        for (int j = 0; j < m; j++) {
          double t = P[col][j]; P[col][j] = P[piv][j]; P[piv][j] = t;
          t = Mi[col][j]; Mi[col][j] = Mi[piv][j]; Mi[piv][j] = t;
        }
      const double p = P[col][col];
      for (int j = 0; j < m; j++) { P[col][j] = P[col][j] / p; Mi[col][j] = Mi[col][j] / p; }
      for (int r = 0; r < m; r++) {
        if (r == col) continue;
        const double f = P[r][col];
        for (int j = 0; j < m; j++) {
          P[r][j] = P[r][j] - f * P[col][j];
          Mi[r][j] = Mi[r][j] - f * Mi[col][j];
        }
      }
    }
    /* the cube: s_j = RU(sum_l |G_jl|) and the room RD(min(c_j - lo_j, hi_j - c_j)) on every axis */
    int e = 0, have = 0;
    for (int j = 0; j < k && ok; j++) {
      const double* I = box + (b * k + j) * 2;
      const double c = centre[(b * k + j) * 2];
      round_up(ORC_OUTWARD);
      double sj = fabs(G[j][0]);
      for (int l = 1; l < m; l++) sj = sj + fabs(G[j][l]);
      round_down(ORC_OUTWARD);
      const double r1 = c - I[0], r2 = I[1] - c;
      round_restore();
      const double room = r1 < r2 ? r1 : r2;
      if (!(sj > 0.0)) continue;
      if (!(room > 0.0)) { ok = 0; break; }
      const int ej = ilogb(room) - ilogb(sj);  /* s 2^ej < 2 room */
      e = have ? (ej < e ? ej : e) : ej;
      have = 1;
    }
    if (!have) ok = 0;
    if (ok) {  /* s_j 2^e <= room_j on every axis, one step down at most */
      int fits = 1;
      for (int j = 0; j < k; j++) {
        const double* I = box + (b * k + j) * 2;
        const double c = centre[(b * k + j) * 2];
        round_up(ORC_OUTWARD);
        double sj = fabs(G[j][0]);
        for (int l = 1; l < m; l++) sj = sj + fabs(G[j][l]);
        round_down(ORC_OUTWARD);
        const double r1 = c - I[0], r2 = I[1] - c;
        round_restore();
        const double room = r1 < r2 ? r1 : r2;
        if (sj > 0.0 && !(ldexp(sj, e) <= room)) fits = 0;
      }
      if (!fits) e -= 1;
    }
    const double r = ok ? ldexp(1.0, e) : 0.0;
    const ivl Y = {-r, r};
    /* A = D G, enclosing phi's Jacobian on Y */
    ivl A[ORC_KMAX][ORC_KMAX];
    for (int q = 0; q < m; q++)
      for (int l = 0; l < m; l++) {
        ivl acc = {0.0, 0.0};
        for (int j = 0; j < k; j++) {
          const double* d = D + (((int64_t)(q * k + j)) * nbox + b) * 2;
          ivl dj = {d[0], d[1]}, g = {G[j][l], G[j][l]};
          ivl t = iv_mul(dj, g, ORC_OUTWARD);
          acc = j == 0 ? t : iv_add(acc, t, ORC_OUTWARD);
        }
        A[q][l] = acc;
      }
    int inside = ok;
    for (int i = 0; i < m; i++) {
      ivl Ki = {0.0, 0.0};
      if (ok) {
        ivl yf = {0.0, 0.0};
        for (int l = 0; l < m; l++) {
          ivl fl = {fc[((int64_t)l * nbox + b) * 2], fc[((int64_t)l * nbox + b) * 2 + 1]};
          ivl ml = {Mi[i][l], Mi[i][l]};
          ivl t = iv_mul(ml, fl, ORC_OUTWARD);
          yf = l == 0 ? t : iv_add(yf, t, ORC_OUTWARD);
        }
        Ki.lo = -yf.hi;
        Ki.hi = -yf.lo;
        for (int l = 0; l < m; l++) {
          ivl a = {i == l ? 1.0 : 0.0, i == l ? 1.0 : 0.0};
          for (int q = 0; q < m; q++) {
            ivl mq = {Mi[i][q], Mi[i][q]};
            ivl t = iv_mul(mq, A[q][l], ORC_OUTWARD);
            ivl nt = {-t.hi, -t.lo};
            a = iv_add(a, nt, ORC_OUTWARD);
          }
          Ki = iv_add(Ki, iv_mul(a, Y, ORC_OUTWARD), ORC_OUTWARD);
        }
        if (!(Ki.lo > -r && Ki.hi < r)) inside = 0;
      }
      if (K) { K[(b * m + i) * 2] = Ki.lo; K[(b * m + i) * 2 + 1] = Ki.hi; }
    }
    if (rout) rout[b] = r;
    out[b] = (uint8_t)inside;
  }
  return 0;
}

int orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
