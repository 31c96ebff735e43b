/*
 * voxcsf.h -- C ABI of libvoxcsf.so: amortized interval subdivision of
 * polynomial systems on MI355X (gfx950).
 *
 * Method: G. Moroz, "Sparse Tensors and Subdivision Methods for Finding the
 * Zero Set of Polynomial Equations", arXiv 2406.09857.
 *   - Sec. 2.1: Compressed Sparse Fiber (CSF) trees; a set of grid boxes is
 *     stored by the indices of its boxes (a tree without leaves values).
 *   - Algorithm 1: Horner's rule on an interval.
 *   - Algorithm 2 (EvaluationCSF) and Theorem 1: evaluation of F on every box
 *     of a CSF by partial evaluation, one variable per tree depth.
 *   - Sec. 3.2, Algorithm 3: subdivision with the exclusion criterion
 *     C0(F, B) = "0 is not in the interval evaluation of F on B"; a system is
 *     excluded on B when any of its polynomials is.
 *
 * Conventions shared by every entry point
 *   - Device pointers are HIP device addresses (e.g. torch CUDA tensors'
 *     data_ptr()); "host" marks host memory.  All device buffers are owned by
 *     the caller; the library keeps no device allocation between calls.
 *   - `stream` is a hipStream_t (NULL = default stream).  Calls enqueue work
 *     on it and return without waiting unless stated otherwise.
 *   - Scratch memory is the caller's `ws` (device, 256-byte aligned: any
 *     other address is VX_EINVAL) of `ws_bytes`; vx_workspace_bytes() gives
 *     the size a call needs.
 *   - Return value: VX_OK or a negative VX_E* code; vx_last_error() then
 *     describes the failure (per host thread).  Argument errors are detected
 *     before anything is enqueued.
 *   - Arithmetic: FP64 intervals, every endpoint rounded outward (lower
 *     endpoints toward -inf, upper toward +inf): a Horner step J*I + C is the
 *     exact range of that set rounded outward once per endpoint (one fused
 *     multiply-add per candidate product), every other operation is rounded
 *     on its own, so {F(x) : x in B} is contained in [lo, hi] for every box
 *     B.  Results are bit-for-bit reproducible (up to the sign of zero
 *     endpoints).
 *   - The domain is a box [dom[2j], dom[2j+1]] per axis j (host array of 2k
 *     finite doubles, dom[2j] < dom[2j+1]).  At level L, axis j is cut into
 *     2^L cells; cell i is enclosed by
 *       [RD(dlo + RD(i * RD(dhi - dlo)) / 2^L), RU(dlo + RU((i+1) * RU(dhi - dlo)) / 2^L)]
 *     which is exact on dyadic domains such as [-1, 1].
 */
#ifndef VOXCSF_H
#define VOXCSF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VX_KMAX 4

enum {
  VX_OK = 0,
  VX_EINVAL = -1,        /* bad argument (null pointer, size, k, degree, domain) */
  VX_ECAPACITY = -2,     /* a caller buffer or the workspace is too small */
  VX_EHIP = -3,          /* a HIP runtime call or kernel launch failed */
  VX_EOVERFLOW = -4,     /* a count or label does not fit in int32 */
  VX_EUNSUPPORTED = -5   /* valid request this build does not implement */
};

/* A polynomial in k variables of total degree <= degree, given as a dense
 * coefficient cube c[e1][e2]...[ek] (C order, side `side` >= degree+1) whose
 * entries with e1+...+ek > degree are ignored.  Coefficients are intervals
 * [c_lo, c_hi]; c_hi == NULL means point coefficients (c_hi = c_lo).  The
 * polynomial CSF of Sec. 2.1 is the simplex support of this cube. */
typedef struct vx_poly {
  int32_t k;
  int32_t degree;
  int32_t side;
  int32_t reserved;
  const double* c_lo;    /* device, side^k doubles */
  const double* c_hi;    /* device, side^k doubles, or NULL */
} vx_poly;

/* A set of boxes of the 2^level grid as a CSF tree (Sec. 2.1).  Depth l+1
 * (l = 0..k-1) holds n[l] nodes; idx[l][q] is the grid index, on axis l, of
 * node q; the children of node q of depth l+1 are the nodes
 * ptr[l][q] .. ptr[l][q+1]-1 of depth l+2 (l < k-1), with strictly ascending
 * labels.  Nodes of one depth are in lexicographic order of their paths, so
 * the depth-k nodes (the boxes, "leaves") are the boxes in lexicographic order.
 * n[l] = N_{l+1}(S) of Definition 1 / Remark 1. */
typedef struct vx_csf {
  int32_t k;
  int32_t level;
  int64_t n[VX_KMAX];    /* host: node counts per depth */
  int64_t cap[VX_KMAX];  /* host: capacity (entries) of idx[l]; ptr[l] holds cap[l]+1 */
  int32_t* idx[VX_KMAX]; /* device labels */
  int32_t* ptr[VX_KMAX]; /* device child offsets, l < k-1 */
} vx_csf;

/* Message describing the last failure on this host thread ("" if none). */
const char* vx_last_error(void);

/* Workspace sizes.  `which` selects the call; arguments not used by that call
 * may be NULL/0.  Returns 0 on invalid arguments. */
enum {
  VX_WS_EVAL = 0,
  VX_WS_FILTER = 1,
  VX_WS_BUILD = 2,
  VX_WS_GRAD = 3,
  VX_WS_MEANVALUE = 4,
  VX_WS_TAYLOR2 = 5,
  VX_WS_INCLUSION = 6,
  VX_WS_NEWTON = 7,
  VX_WS_ORDER = 8
};
size_t vx_workspace_bytes(int32_t which, const vx_poly* P, int32_t np, const vx_csf* S, int64_t n);

/*
 * csf_build -- CSF of an arbitrary list of boxes (Sec. 2.1).
 *   boxes : device int32, n x k row-major grid indices in [0, 2^level), any
 *           order, duplicates allowed (they are merged).
 *   out   : caller CSF with k, level set and idx/ptr of capacity >= n at every
 *           depth; on return out->n[] holds the node counts (this call waits
 *           for the stream to read them back).
 * Errors: VX_EINVAL (k, level, negative n, labels outside the grid are
 * reported as VX_EINVAL after the build), VX_ECAPACITY (out->cap < n, ws).
 */
int csf_build(int32_t k, int32_t level, const int32_t* boxes, int64_t n, vx_csf* out, void* ws, size_t ws_bytes,
              void* stream);

/*
 * interval_eval_level -- Algorithm 2 on one level: enclosures of np
 * polynomials (one system: same k) on every box of S.
 *   lo, hi : device double, np x S->n[k-1], row p = polynomial p, boxes in
 *            CSF leaf order.
 *   keep   : device uint8, S->n[k-1], or NULL: keep[b] = 1 unless some
 *            polynomial's enclosure on box b excludes 0 (lo > 0 or hi < 0);
 *            NaN endpoints never exclude.  This is criterion C0 over the
 *            system.
 * The amortization follows Theorem 1: the polynomial is partially evaluated
 * at each depth-1 interval once, the result at each depth-2 interval once,
 * and so on; the work is sum_l (Nt_{k-l} - Nt_{k-l-1}) N_{l+1}(S) interval
 * Horner steps per polynomial (Nt_m = C(d+m, m)).
 * Errors: VX_EINVAL (k mismatch, degree/side, null pointers, domain),
 * VX_ECAPACITY (ws smaller than vx_workspace_bytes(VX_WS_EVAL, ...)).
 */
int interval_eval_level(const vx_poly* P, int32_t np, const vx_csf* S, const double* dom, double* lo, double* hi,
                        uint8_t* keep, void* ws, size_t ws_bytes, void* stream);

/*
 * interval_eval_level_noalloc -- interval_eval_level without a workspace
 * argument, for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * scratch is a static 64 MiB device array of the library, one per GPU, held
 * until the process ends; the call itself allocates nothing.
 *   Arguments, outputs, results (bit for bit) and errors as
 *   interval_eval_level; the caller still passes the inputs and outputs.
 *   A level whose vx_workspace_bytes(VX_WS_EVAL, ...) exceeds 64 MiB
 *   (67,108,864 bytes) is refused with VX_ECAPACITY before anything is
 *   enqueued.
 *   Every call on one GPU shares that GPU's array, and the array keeps the
 *   last call's contents (every call rewrites what it reads): calls that
 *   overlap on one GPU (other host threads, or other streams whose work has
 *   not finished) race and give undefined results.  The first call on a
 *   device looks up the array's device address once (hipGetSymbolAddress).
 */
int interval_eval_level_noalloc(const vx_poly* P, int32_t np, const vx_csf* S, const double* dom, double* lo,
                                double* hi, uint8_t* keep, void* stream);

/*
 * mean_value_exclusion -- the Taylor form of order 1 (Sec. 3.2, Taylor form
 * definition with m = 1) as an exclusion test on every box of S:
 *   T(F_p, B) = F_p(c) + sum_i dF_p/dx_i(B) * (B_i - c_i),  c the centre of B,
 * each part an outward-rounded enclosure computed by Algorithm 2 on S: F_p at
 * the degenerate boxes of the centre enclosures (the centre of cell i at
 * level L is the common endpoint of cells 2i, 2i+1 at level L+1), the
 * derivative polynomials (coefficients (e_i+1) c_{e+u_i}, rounded outward) on
 * the boxes, B_i - c_i = [RD(lo_i - chi_i), RU(hi_i - clo_i)], and the sum
 * left to right over i.  {F_p(x) : x in B} is contained in T(F_p, B).
 *   lo, hi : device double, np x S->n[k-1], the mean-value enclosures.
 *   keep   : device uint8 or NULL; if given, keep[b] is cleared when some
 *            T(F_p, B) excludes 0 (AND with the caller's flags, e.g. C0's).
 * Limits: np * k <= 64.  Errors as interval_eval_level; workspace
 * vx_workspace_bytes(VX_WS_MEANVALUE, P, np, S, 0).
 */
int mean_value_exclusion(const vx_poly* P, int32_t np, const vx_csf* S, const double* dom, double* lo, double* hi,
                         uint8_t* keep, void* ws, size_t ws_bytes, void* stream);

/* Highest order of the Taylor forms (taylor_exclusion, VX_RUN_TAYLOR_ORDER). */
#define VX_TAYLOR_MAX_ORDER 6

/*
 * taylor_exclusion -- the Taylor form of order `order` (1..VX_TAYLOR_MAX_ORDER;
 * Sec. 3.2, Taylor form definition) as an exclusion test on every box of S.
 * Order 1 is mean_value_exclusion.  Order 2:
 *   T2(F_p, B) = F_p(c) + sum_i dF_p/dx_i(c) W_i + sum_{i<=j} H_ij(B) X_ij,
 * W_i = B_i - c_i = [RD(lo_i - chi_i), RU(hi_i - clo_i)] (c's enclosure as in
 * mean_value_exclusion), H_ii = (1/2) d2F_p/dx_i^2 and H_ij = d2F_p/dx_i dx_j
 * (i < j), whose coefficients m c_{e+u_i+u_j} (m = (e_i+1)(e_i+2)/2 or
 * (e_i+1)(e_j+1), an exact integer) are rounded outward once, X_ii the range
 * of the square ([0, RU(max(a^2, b^2))] for W_i = [a, b] holding 0) and
 * X_ij = W_i W_j.  F_p and its gradient are evaluated at the centre
 * enclosures and the H_ij on the boxes, each by Algorithm 2 on S; the terms
 * are added left to right, gradient terms first, then the pairs in
 * lexicographic order.  {F_p(x) : x in B} is contained in T2(F_p, B).
 *   lo, hi : device double, np x S->n[k-1], the order-`order` enclosures.
 *   keep   : device uint8 or NULL; if given, keep[b] is cleared when some
 *            enclosure excludes 0 (AND with the caller's flags).
 * Order m >= 3, in the multinomial form of the definition:
 *   T_m(F_p, B) = F_p(c) + sum_{t >= 1} T_t X_t
 * over the multi-indices alpha_t of orders 1..m: orders in increasing
 * order, each order's multi-indices as the non-decreasing index tuples
 * i_1 <= ... <= i_j in lexicographic order (for m = 2 this is the sum
 * above).  T_t is the coefficient polynomial D^alpha F_p / alpha!, whose
 * coefficients prod_i C(e_i + alpha_i, alpha_i) c_{e + alpha} (an exact
 * integer times c) are rounded outward once, evaluated at the centre
 * enclosures for orders below m and over the box for order m, each by
 * Algorithm 2 on S; X_t = prod_i W_i^(alpha_i) with W_i = B_i - c_i as above
 * and each power the range of x^a over W_i ([-RU(|lo|^a), RU(hi^a)] for odd
 * a, [0, RU(max(|lo|, hi)^a)] for even a, powers formed by repeated
 * multiplication), the powers multiplied over ascending i; the terms are
 * added left to right.  {F_p(x) : x in B} is contained in T_m(F_p, B).
 * Limits: np * k <= 64 (order 1), np * k(k+1)/2 <= 64 (order 2); any np for
 * m >= 3 (its term systems are cut into groups of 64); C(degree + m, m) <
 * 2^53 (VX_EUNSUPPORTED otherwise).  Errors as interval_eval_level,
 * VX_EINVAL for an order outside 1..VX_TAYLOR_MAX_ORDER; workspace
 * vx_taylor_workspace_bytes(P, np, S, order) (for orders 1 and 2 also
 * vx_workspace_bytes(VX_WS_MEANVALUE or VX_WS_TAYLOR2, P, np, S, 0)).
 */
int taylor_exclusion(const vx_poly* P, int32_t np, const vx_csf* S, const double* dom, int32_t order, double* lo,
                     double* hi, uint8_t* keep, void* ws, size_t ws_bytes, void* stream);
/* Workspace of taylor_exclusion of that order on S (0 on invalid arguments). */
size_t vx_taylor_workspace_bytes(const vx_poly* P, int32_t np, const vx_csf* S, int32_t order);

/*
 * inclusion_test -- the inclusion criterion C1 of Sec. 3.2 ("Inclusion
 * Criterion") on every box of S and every polynomial: F_p on the 2^k
 * vertices of the box, the box certified when one vertex enclosure has a
 * lower bound > 0 and another an upper bound < 0 (then F_p vanishes in the
 * box, by the intermediate value theorem).  Vertex v of the 2^level grid on
 * an axis is enclosed by [lower end of cell v, upper end of cell v-1] (exact
 * on dyadic domains).  The vertices of all boxes form a subset of the vertex
 * grid: they are evaluated once each by Algorithm 2 on their own CSF
 * (built on the device with the csf_build sort), as the paper suggests.
 *   incl : device uint8, np x S->n[k-1], row p = polynomial p, boxes in CSF
 *          leaf order; 1 = certified, 0 = not certified.  NaN bounds certify
 *          nothing.
 * The call waits for the stream once (the vertex count sizes the
 * evaluation).  Limits: k * (level + 1) <= 62.  Errors as
 * interval_eval_level, VX_EUNSUPPORTED beyond the limit; workspace
 * vx_workspace_bytes(VX_WS_INCLUSION, P, np, S, 0).
 */
int inclusion_test(const vx_poly* P, int32_t np, const vx_csf* S, const double* dom, uint8_t* incl, void* ws,
                   size_t ws_bytes, void* stream);

/*
 * taylor_inclusion_test -- the inclusion criterion C1 from the order-2 Taylor
 * form (Sec. 3.2, "Inclusion Criterion", Taylor variant): the linear part
 * l(x) = F_p(c) + grad F_p(c).(x - c) is largest at the vertex V_max that
 * takes, on axis i, the box's upper end when the enclosure [a, b] of
 * dF_p/dx_i(c) has a + b >= 0 and the lower end otherwise, and smallest at
 * the opposite vertex V_min; F_p at a vertex V is bounded by the order-2 form
 * at the point V (taylor_exclusion's sum with V_i - c_i in place of B_i - c_i,
 * from the vertex enclosures of inclusion_test and H_ij still over B).  The
 * box is certified when the lower bound at V_max is > 0 and the upper bound
 * at V_min is < 0.
 *   incl : device uint8, np x S->n[k-1], as inclusion_test.
 * Limits, errors and workspace as taylor_exclusion with order 2
 * (vx_workspace_bytes(VX_WS_TAYLOR2, ...)).
 */
int taylor_inclusion_test(const vx_poly* P, int32_t np, const vx_csf* S, const double* dom, uint8_t* incl, void* ws,
                          size_t ws_bytes, void* stream);

/*
 * newton_test -- the Newton interval inclusion test for a system of
 * 1 <= np <= k polynomials (Sec. 3.2, inclusion criterion for several
 * polynomials), on every box of S.
 *
 * Square systems (np == k), in Krawczyk's form:
 *   K(B) = c - Y F(c) + (I - Y S)(B - c),
 * c the centre enclosure, S the slope matrix of the box (S_ij enclosed by
 * dF_i/dx_j on the box with x_1..x_j free and x_{j+1}..x_k at the centre,
 * each column one Algorithm-2 evaluation with cells on the first j axes and
 * centres on the others), Y = (mid S)^-1 in round-to-nearest (mid =
 * (lo + hi) * 0.5, Gauss-Jordan with partial pivoting: first largest
 * |pivot|, pivot row divided by the pivot, r -= f * pivot row), K in outward
 * arithmetic with every sum in ascending index order.  The box is certified
 * (F has a zero in it) when every K_i lies in the inner box [upper end of
 * the lower vertex enclosure, lower end of the upper one]; a zero pivot
 * certifies nothing.
 *
 * Fewer polynomials than variables (np = m < k; the same passage: the box
 * intersected with the span of the gradients at its centre gives a square
 * system): with c the lower end of the centre enclosure and G (k x m) the
 * midpoints of the gradient enclosures at the centre (column l for F_l),
 * phi(y) = F(c + G y) is tested on the cube Y = [-r, r]^m, r the largest
 * power of two with s_j r <= min(c_j - lo_j, hi_j - c_j) on every axis
 * (s_j = sum_l |G_jl| rounded up, the room rounded down), so that c + G Y
 * lies in the box:
 *   K(Y) = -M phi(0) + (I - M A) Y,   A = D G,   M = (mid(D) G)^-1,
 * D the gradients enclosed on the box (one Algorithm-2 evaluation of the
 * derivative polynomials), phi(0) enclosed by F on the centre enclosure;
 * G, mid(D) G and M in round-to-nearest, K outward, sums in ascending index
 * order.  K inside the open cube certifies a zero of F in the box.
 *
 *   incl : device uint8, S->n[k-1]; 1 = certified.
 *   kout : device double, S->n[k-1] x np x 2 (box, component, lo/hi), or
 *          NULL: K (in the cube's coordinates when np < k).
 * Errors as interval_eval_level, VX_EINVAL when np > k; workspace
 * vx_workspace_bytes(VX_WS_NEWTON, P, np, S, 0).
 */
int newton_test(const vx_poly* P, int32_t np, const vx_csf* S, const double* dom, uint8_t* incl, double* kout,
                void* ws, size_t ws_bytes, void* stream);

/*
 * variable_order_costs -- Theorem 1's cost of evaluating S under several
 * orders of the variables (Theorem 1, Sec. 1 "Main Result": the cost sums
 * the trailing-tuple counts times the node counts N_l(S), and the node
 * counts depend on which variable each CSF depth holds).  Order o lists,
 * for each CSF depth l, the axis a = orders[o*k + l] that depth holds (the
 * default order is 0, 1, ..., k-1); its node counts are those of the CSF of
 * S's boxes with their labels listed in that order, built on the device.
 *   orders : host int32, norders x k, each a permutation of 0..k-1
 *            (1 <= norders <= 24; VX_EINVAL otherwise).
 *   counts : host int64, norders x k, the node counts N_1..N_k (or NULL).
 *   steps  : host int64, norders, the interval Horner steps of Theorem 1 for
 *            the dense total-degree polynomials P (their degrees only; a
 *            permuted dense simplex is one of the same degree) (or NULL;
 *            P may then be NULL).
 * Runs the evaluation with the chosen order by transposing every
 * polynomial's coefficients the same way (new variable l = old variable
 * orders[o*k + l]).  Synchronous; VX_EUNSUPPORTED when k * level > 62;
 * workspace vx_workspace_bytes(VX_WS_ORDER, NULL, 0, S, 0).
 */
int variable_order_costs(const vx_poly* P, int32_t np, const vx_csf* S, int32_t norders, const int32_t* orders,
                         int64_t* counts, int64_t* steps, void* ws, size_t ws_bytes, void* stream);

/*
 * filter_subdivide -- exclusion filter and bisection (Algorithm 3): prune S
 * to the kept boxes K (keep[b] != 0, internal nodes without kept descendants
 * removed) and build the CSF of their 2^k children at level+1, child c of box
 * B being 2B + c, c in {0,1}^k (bisection of G_n into G_2n, Sec. 3.2).
 *   keep     : device uint8, S->n[k-1].
 *   kept     : caller CSF, cap[l] >= S->n[l]; may be NULL (not written).
 *   next     : caller CSF, cap[l] >= 2^(l+1) S->n[l]; may be NULL.
 *   d_counts : device int64[2k]: K's n[0..k-1] then next's n[0..k-1].
 * The host-side n[] of kept/next are not updated (the counts are on the
 * device); copy d_counts back before using them.
 * Errors: VX_EINVAL, VX_ECAPACITY (caps below the bounds above, ws).
 */
int filter_subdivide(const vx_csf* S, const uint8_t* keep, vx_csf* kept, vx_csf* next, int64_t* d_counts, void* ws,
                     size_t ws_bytes, void* stream);

/* Per-level record of run_subdivision. */
typedef struct vx_level_stat {
  int32_t level;
  int32_t axes;           /* variable order of the run: CSF depth l holds axis (axes >> 4l) & 15 */
  int64_t n[VX_KMAX];     /* N_l of the evaluated set S_level */
  int64_t kept[VX_KMAX];  /* N_l of the kept set K_level */
  int64_t steps;          /* interval Horner steps, all polynomials (Theorem 1 count) */
  double eval_ms;         /* interval_eval_level time (HIP events) */
  double filter_ms;       /* filter_subdivide time (HIP events) */
  int64_t certified;      /* boxes certified by C1 at this level (VX_RUN_INCLUSION*) */
} vx_level_stat;

/* Called after each level with device pointers valid until it returns; a
 * nonzero return stops the run (VX_OK is still returned). */
typedef int (*vx_level_cb)(void* user, int32_t level, const vx_csf* S, const double* lo, const double* hi,
                           const uint8_t* keep, const vx_csf* kept);

/*
 * run_subdivision -- Algorithm 3 with C0 only, from the whole domain (level
 * 0) to level `depth`: evaluate, filter, bisect, repeat.  The boxes kept at
 * the last level are the enclosure of the zero set.
 *   stats : host array of depth+1 records (may be NULL).
 *   cb    : optional per-level callback.
 *   ws    : one device workspace carved into all level buffers; if it is too
 *           small the call returns VX_ECAPACITY and *ws_needed (if not NULL)
 *           receives a sufficient size for the level that did not fit.
 * The call synchronizes the stream once per level (to read the counts).
 */
int run_subdivision(const vx_poly* P, int32_t np, const double* dom, int32_t depth, void* ws, size_t ws_bytes,
                    size_t* ws_needed, vx_level_stat* stats, vx_level_cb cb, void* user, void* stream);

/* run_subdivision with options.  flags: VX_RUN_MEAN_VALUE adds the
 * mean-value test (mean_value_exclusion) to C0 at every level: a box is kept
 * only when both tests keep it (eval_ms then includes both; the callback
 * still receives the C0 enclosures and the combined keep flags).
 * VX_RUN_TAYLOR2 adds the order-2 Taylor test (taylor_exclusion, order 2) in
 * the same way, VX_RUN_TAYLOR_ORDER(m) the Taylor test of order m
 * (1..VX_TAYLOR_MAX_ORDER); these flags are exclusive (VX_EINVAL).  VX_RUN_NO_TIMES
 * records no per-level timing events (stats eval_ms and filter_ms are 0):
 * each event is a packet the stream must pass between the level's kernels.
 * VX_RUN_INCLUSION (C1: vertex signs, inclusion_test, for one polynomial;
 * the Newton test, newton_test, for a system of 2..k polynomials) or
 * VX_RUN_INCLUSION_TAYLOR (the Taylor form of the vertex test,
 * taylor_inclusion_test, one polynomial), with VX_RUN_INCLUSION_FROM(L), run
 * Algorithm 3 with both criteria: from level L on (boxes smaller than the
 * threshold) the boxes kept by C0 that C1 certifies join the output and are
 * not bisected; stats certified counts them, the callback sees keep = 2 for
 * them (1: continue, 0: excluded) and K holds the continuing boxes.
 * VX_EINVAL for other systems and for both inclusion flags.
 * VX_RUN_EARLY_EXIT (systems, np >= 2; Sec. 3.2: a box is excluded as soon
 * as one polynomial excludes it) evaluates polynomial p only on the boxes
 * that polynomials 0..p-1 kept, compacting the survivors after each one; the
 * kept sets, and so the whole run, are those of the plain loop.  stats steps
 * counts the steps actually spent, eval_ms includes the compactions, and the
 * callback receives lo = hi = keep = NULL (they cover subsets of S).  Each
 * compaction costs a filter pass and a wait for its counts, which only large
 * levels repay: with VX_RUN_EARLY_EXIT_FROM(L) the levels below L are
 * evaluated as without the flag.  It does not combine with the Taylor or
 * inclusion flags (VX_EINVAL); with one polynomial it has no effect.
 * VX_RUN_AUTO_ORDER picks the order of the variables by Theorem 1 (its cost
 * sums the trailing-tuple counts times the node counts N_l(S), which depend on
 * which variable each CSF depth holds): a probe run in the given order to
 * level L (VX_RUN_AUTO_ORDER_AT(L), 1..15, default min(depth, 6); plain C0, no
 * timing) gives the evaluated set of level L, its node counts are taken under
 * all k! orders (as variable_order_costs does), and the whole run (levels
 * 0..depth, with the other flags) is done in the cheapest order, ties going
 * to the first order in lexicographic order of the permutations (the given
 * order first).  The run in order sigma is the run of the polynomials with
 * new variable l = old variable sigma[l] (coefficient cubes transposed, the
 * domain's axes permuted): every CSF passed to the callback lists its labels
 * in that order, and stats[].axes records it.  The probe adds the cost of
 * levels 0..L; workspace as without the flag plus the transposed coefficients
 * and the order scratch (run_subdivision_ex reports the total in *ws_needed). */
enum {
  VX_RUN_MEAN_VALUE = 1,
  VX_RUN_TAYLOR2 = 2,
  VX_RUN_NO_TIMES = 4,
  VX_RUN_INCLUSION = 8,
  VX_RUN_INCLUSION_TAYLOR = 16,
  VX_RUN_EARLY_EXIT = 32,
  VX_RUN_AUTO_ORDER = 64
};
#define VX_RUN_TAYLOR_ORDER(m) ((int32_t)(m) << 8)
#define VX_RUN_AUTO_ORDER_AT(level) ((int32_t)(level) << 12)
#define VX_RUN_INCLUSION_FROM(level) ((int32_t)(level) << 16)
#define VX_RUN_EARLY_EXIT_FROM(level) ((int32_t)(level) << 24)
int run_subdivision_ex(const vx_poly* P, int32_t np, const double* dom, int32_t depth, int32_t flags, void* ws,
                       size_t ws_bytes, size_t* ws_needed, vx_level_stat* stats, vx_level_cb cb, void* user,
                       void* stream);

/* Copy `bytes` between host and device or device and device on `stream` and
 * wait for it (helper for callbacks). kind: 0 = device->host, 1 = host->device,
 * 2 = device->device. */
int vx_copy(void* dst, const void* src, size_t bytes, int32_t kind, void* stream);

/*
 * eval_grad -- point values and gradients of a polynomial system, and the
 * gradient of sum_{p,i} gbar[p][i] F_p(x_i) with respect to the coefficients
 * (the adjoint of the evaluation).  Round-to-nearest FP64: values by nested
 * Horner in the order of the interval path (x1 innermost) with no fused
 * multiply-add, so f is bit-identical to that plain evaluation; derivatives
 * are carried forward along the same chains, each step one fused
 * multiply-add (the same with and without a grid).  Sec. 3.2 uses the gradients for
 * Newton steps in the span of the gradients and for Taylor forms.
 *   P, np  : point coefficients (c_hi must be NULL), np <= 4, same k.
 *   x      : device, n x k points (row-major).
 *   f      : device, np x n values, or NULL.
 *   jac    : device, n x np x k partial derivatives dF_p/dx_j, or NULL.
 *   gbar   : device, np x n weights, or NULL.
 *   xbar   : device, n x k, or NULL: sum_p gbar[p][i] dF_p/dx_j (x_i), the
 *            gradient of the weighted sum with respect to the points.
 *   dcoef  : device, np dense cubes (side^k each, zeros outside the simplex)
 *            receiving sum_i gbar[p][i] x_i^e; requires `grid`.
 *   grid, dom : the points are the centres of the leaves of this CSF on the
 *            domain dom (host, 2k), in leaf order (n = grid->n[k-1]), or
 *            grid = NULL for arbitrary points.  With a grid, f and jac come
 *            from the amortized evaluation of Algorithm 2 with points for
 *            boxes: each partial evaluation is computed once per CSF node and
 *            shared by all points below it (Sec. 1.1, Property 1; Theorem 1),
 *            bit-identical to the per-point evaluation; and the coefficient
 *            gradient is the transpose of that evaluation, one CSF depth at a
 *            time.  x may then be NULL; if it is given, it must equal the
 *            centres as csf_centres writes them, bit for bit (checked on the
 *            device, the call then waits for the stream once; VX_EINVAL
 *            otherwise).
 * Errors: VX_EINVAL, VX_EUNSUPPORTED (dcoef without grid; degree > 200 for
 * dcoef), VX_ECAPACITY (workspace: vx_workspace_bytes(VX_WS_GRAD, P, np,
 * grid, n)).
 */
int eval_grad(const vx_poly* P, int32_t np, const double* x, int64_t n, double* f, double* jac, const double* gbar,
              double* xbar, double* dcoef, const vx_csf* grid, const double* dom, void* ws, size_t ws_bytes,
              void* stream);

/* csf_centres -- centres of the cells of the leaves of S on the domain (host
 * dom[2k]), device output n[k-1] x k, leaf order; round-to-nearest (exact on
 * dyadic domains). */
int csf_centres(const vx_csf* S, const double* dom, double* x, void* stream);

/*
 * newton_project -- `steps` Newton steps x <- x - J^T (J J^T)^{-1} F(x) on
 * every point (the minimum-norm step in the span of the gradients, Sec. 3.2,
 * for systems with fewer equations than unknowns; J is np x k).  Points whose
 * J J^T is singular are left in place.  x (device, n x k) is updated in
 * place; f (device np x n, or NULL) receives F at the final points.
 */
int newton_project(const vx_poly* P, int32_t np, double* x, int64_t n, int32_t steps, double* f, void* ws,
                   size_t ws_bytes, void* stream);

/*
 * newton_project_grid -- newton_project from the centres of a CSF's leaves
 * (x, n = grid->n[k-1] points in leaf order, as csf_centres writes them, on
 * the domain dom): the first evaluation of F and J, at those centres, runs
 * on the CSF grid by Algorithm 2 (Sec. 1.1, Property 1: each coordinate
 * paid once per fiber) instead of per point; the later steps leave the grid
 * and evaluate per point.  Results are bit-identical to newton_project.  x
 * must equal the centres bit for bit (checked on the device; VX_EINVAL
 * otherwise, x unchanged).  Workspace: vx_workspace_bytes(VX_WS_GRAD, P, np,
 * grid, n).
 */
int newton_project_grid(const vx_poly* P, int32_t np, double* x, int64_t n, int32_t steps, double* f,
                        const vx_csf* grid, const double* dom, void* ws, size_t ws_bytes, void* stream);

/*
 * Batched subdivision -- many independent systems run through Algorithm 3 in
 * lockstep (all levels 0..depth), for workloads of many small problems where
 * one system cannot fill the GPU.  Batching independent systems is this
 * library's own design, not the paper's (whose only remark on parallelism,
 * in Sec. 4.1, is that its CPU implementation can spread one computation
 * over several threads): every kernel covers all systems at once.
 *
 * The box sets of all systems form one CSF with an extra top depth: depth 0
 * holds one node per live system (label = system index), depths 1..k hold the
 * grid indices as in vx_csf.  Every count stays on the device and every
 * kernel is a fixed-shape persistent grid-stride loop, so one run is a fixed
 * launch sequence that can be captured once as a HIP graph and replayed.
 * Each system's boxes, enclosures and keep flags are bit-identical to
 * run_subdivision on that system alone (same arithmetic in the same order).
 *
 * Scope: k = 3 and one polynomial per system (C0 on a single equation),
 * 1 <= nsys <= 64, one domain for all systems.
 *
 *   cap   : host int64[k+1], node capacity per depth of the batched CSF
 *           (cap[0] >= nsys).  A run that would exceed it stops growing,
 *           finishes with empty levels, and vx_batch_result reports
 *           VX_ECAPACITY together with the counts it needed.
 *   tune  : host array of depth+1 launch configurations (one per level), or
 *           NULL for defaults: r1 = depth-1 nodes per stage-1 wave (1, 2, 4
 *           or 8), groups = chain groups per middle-stage segment (1..64),
 *           grid = workgroups of the evaluation kernels (64..65536).
 *           The configuration changes the work distribution only, never a
 *           result.
 *   flags : VX_BATCH_GRAPH = capture the run as a HIP graph on the first
 *           vx_batch_run and replay it afterwards (captured on a private
 *           stream, launched on the caller's).
 *   ws    : device workspace of vx_batch_workspace_bytes(P, nsys, depth, cap)
 *           bytes, owned by the caller, used by the handle until
 *           vx_batch_destroy.  The coefficient buffers of P are read by every
 *           run (the tables are rebuilt at the start of each run).
 * The handle holds host state only (configuration, graph); it is not
 * thread-safe, and runs of one handle must not overlap.
 */
typedef struct vx_batch vx_batch;
typedef struct vx_batch_tune {
  int32_t r1;
  int32_t groups;
  int32_t grid;
  int32_t reserved;
} vx_batch_tune;
enum { VX_BATCH_GRAPH = 1 };

size_t vx_batch_workspace_bytes(const vx_poly* P, int32_t nsys, int32_t depth, const int64_t* cap);
int vx_batch_create(const vx_poly* P, int32_t nsys, const double* dom, int32_t depth, const int64_t* cap,
                    const vx_batch_tune* tune, int32_t flags, void* ws, size_t ws_bytes, void* stream,
                    vx_batch** out);
/* Enqueue one whole run (levels 0..depth) on `stream`; does not wait. */
int vx_batch_run(vx_batch* b, void* stream);
/* Per-level record of a batched run, summed over systems: node counts of
 * the evaluated and of the kept set per batched depth (0 = live systems,
 * l = 1..k as in vx_csf), and the interval Horner steps of Theorem 1, per
 * CSF depth of the systems (steps_depth[l], l = 0..k-1) and in total. */
typedef struct vx_batch_stat {
  int32_t level;
  int32_t reserved;
  int64_t n[VX_KMAX];
  int64_t kept[VX_KMAX];
  int64_t steps;
  int64_t steps_depth[VX_KMAX];
} vx_batch_stat;
/* Wait for the stream, then report the last run:
 *   stats : host array of depth+1 records, or NULL.
 *   need  : host int64[k+1] or NULL: the largest node counts per depth the
 *           run reached (a sufficient `cap` after VX_ECAPACITY, as far as the
 *           run got).
 *   last  : batched CSF (k+1 depths, caps >= counts) receiving the evaluated
 *           set of the last level, or NULL; lo/hi/keep: device arrays of its
 *           leaves' enclosures and keep flags, or NULL.
 *   kept  : batched CSF receiving the kept set of the last level, or NULL. */
int vx_batch_result(vx_batch* b, vx_batch_stat* stats, int64_t* need, vx_csf* last, double* lo, double* hi, uint8_t* keep,
                    vx_csf* kept, void* stream);
/* Autotuner: run every candidate configuration `reps` times eagerly, and
 * keep per level the fastest (written to chosen[depth+1] and its time to
 * level_ms[depth+1], either may be NULL).  Waits for the stream. */
int vx_batch_autotune(vx_batch* b, const vx_batch_tune* cand, int32_t ncand, int32_t reps, vx_batch_tune* chosen,
                      float* level_ms, void* stream);
void vx_batch_destroy(vx_batch* b);

/* Per-kernel timing.  vx_profile_begin() starts recording HIP events around
 * every evaluation and filter kernel launched afterwards from any host thread;
 * vx_profile_end() waits for the recorded events, fills up to `max` records
 * (one per kernel name: launches, total milliseconds, and the algorithmic
 * work units of those launches -- interval Horner steps for the evaluation
 * kernels, elements for the filter kernels), stores the number of names in
 * *count and stops recording. */
typedef struct vx_kernel_stat {
  char name[32];
  int64_t launches;
  double ms;
  double units;
} vx_kernel_stat;
int vx_profile_begin(void);
int vx_profile_end(vx_kernel_stat* out, int32_t max, int32_t* count);
/* Restrict later recording to the launches of one kernel name (NULL or ""
 * records every kernel again), so that a timed run pays for two event
 * records per launch of that kernel only.  VX_EINVAL for names of 32 or more
 * characters. */
int vx_profile_select(const char* name);

#ifdef __cplusplus
}
#endif

#endif /* VOXCSF_H */
