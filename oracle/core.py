"""Python side of the oracle -- TEST INFRASTRUCTURE ONLY.

ctypes wrapper around ``liboracle.so`` (oracle.c) plus the plain numpy
bookkeeping of the subdivision loop: building a box CSF from a set of grid
indices, the exclusion test and the bisection.  Only tests, the smoke check
and the benchmark's CPU-baseline leg use this module.

Paper: G. Moroz, arXiv 2406.09857.
  * CSF of a set of grid indices: Sec. 2.1 (labelled tree; the children of a
    depth-l node are the projections pi_t(E)); Remark 1 (N_i = number of
    depth-i nodes).
  * Algorithm 2 (EvaluationCSF) and Theorem 1: ``eval_csf``.
  * Algorithm 3 (subdivision) restricted to the exclusion criterion C0 and a
    fixed depth: ``subdivide``.  C0(F, B) is "0 not in []F(B)" (Sec. 3.2); a
    system is excluded when any of its polynomials excludes 0.
  * The Taylor form of Sec. 3.2 as an exclusion test: order 1 (the mean-value
    form, ``mean_value_level``, ``subdivide_mv``), order 2
    (``taylor2_level``, ``subdivide_t2``) and any order m
    (``taylor_m_level``, ``subdivide_tm``).
  * The inclusion criterion C1 of Sec. 3.2 (sign change over the vertices of
    a box, the vertices evaluated by Algorithm 2 on their grid):
    ``inclusion_level``; for square systems the Newton interval test
    (Krawczyk's form, slopes by Algorithm 2 on mixed box/centre grids):
    ``newton_level``.
"""
from __future__ import annotations

import ctypes as C
import itertools
import math
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC_PATH = os.path.join(HERE, "oracle.c")

OUTWARD = 0
NEAREST = 1


def build(force: bool = False) -> str:
    """Compile liboracle.so with a strict floating-point model (clang)."""
    if not force and os.path.exists(LIB_PATH) and os.path.getmtime(LIB_PATH) >= os.path.getmtime(SRC_PATH):
        return LIB_PATH
    clang = "/opt/rocm/llvm/bin/clang"
    if not os.path.exists(clang):
        clang = "clang"
    cmd = [clang, "-O2", "-ffp-model=strict", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
           "-Wall", "-o", LIB_PATH + ".tmp", SRC_PATH, "-lm", "-Wl,-rpath,/opt/rocm/llvm/lib"]
    subprocess.check_call(cmd)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB_PATH)
        dp = C.POINTER(C.c_double)
        i64p = C.POINTER(C.c_int64)
        L.orc_iv_add.argtypes = [dp, dp, C.c_int, dp]
        L.orc_iv_mul.argtypes = [dp, dp, C.c_int, dp]
        L.orc_iv_muladd.argtypes = [dp, dp, dp, C.c_int, dp]
        L.orc_box.argtypes = [C.c_double, C.c_double, C.c_int, C.c_int64, dp]
        L.orc_box_table.argtypes = [C.c_double, C.c_double, C.c_int, C.c_int64, dp]
        L.orc_eval_box.argtypes = [C.c_int, C.c_int, C.c_int, dp, dp, dp, C.c_int, dp, i64p]
        L.orc_eval_box.restype = C.c_int
        L.orc_eval_csf.argtypes = [C.c_int, C.c_int, C.c_int, dp, dp, i64p,
                                   C.POINTER(C.POINTER(C.c_int32)), C.POINTER(C.POINTER(C.c_int32)),
                                   C.POINTER(dp), i64p, C.c_int, C.c_int, dp, dp, i64p]
        L.orc_eval_csf.restype = C.c_int
        L.orc_eval_points.argtypes = [C.c_int, C.c_int, C.c_int, dp, dp, C.c_int64, dp]
        L.orc_eval_points.restype = C.c_int
        L.orc_max_threads.restype = C.c_int
        L.orc_centre_table.argtypes = [C.c_double, C.c_double, C.c_int, C.c_int64, dp]
        L.orc_deriv.argtypes = [C.c_int, C.c_int, C.c_int, dp, dp, C.c_int, dp, dp]
        L.orc_deriv.restype = C.c_int
        L.orc_mean_value.argtypes = [C.c_int, C.c_int64, dp, dp, dp, dp, dp]
        L.orc_mean_value.restype = C.c_int
        L.orc_vertex_table.argtypes = [C.c_double, C.c_double, C.c_int, C.c_int64, dp]
        L.orc_vertex_table.restype = None
        L.orc_taylor_inclusion.argtypes = [C.c_int, C.c_int64, dp, dp, dp, dp, dp, dp,
                                           np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")]
        L.orc_taylor_inclusion.restype = C.c_int
        L.orc_krawczyk.argtypes = [C.c_int, C.c_int64, dp, dp, dp, dp, dp,
                                   np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS"), dp]
        L.orc_krawczyk.restype = C.c_int
        L.orc_newton_span.argtypes = [C.c_int, C.c_int, C.c_int64, dp, dp, dp, dp, dp,
                                      np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS"), dp, dp]
        L.orc_newton_span.restype = C.c_int
        L.orc_deriv2.argtypes = [C.c_int, C.c_int, C.c_int, dp, dp, C.c_int, C.c_int, dp, dp]
        L.orc_deriv2.restype = C.c_int
        L.orc_taylor2.argtypes = [C.c_int, C.c_int64, dp, dp, dp, dp, dp, dp]
        L.orc_taylor2.restype = C.c_int
        i32p = C.POINTER(C.c_int32)
        L.orc_taylor_coef.argtypes = [C.c_int, C.c_int, C.c_int, dp, dp, i32p, dp, dp]
        L.orc_taylor_coef.restype = C.c_int
        L.orc_taylor_m.argtypes = [C.c_int, C.c_int, i32p, C.c_int64, dp, dp, dp, dp]
        L.orc_taylor_m.restype = C.c_int
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def max_threads() -> int:
    return int(lib().orc_max_threads())


# ---------------------------------------------------------------------------
# Primitive operations
# ---------------------------------------------------------------------------

def iv_add(x, y, mode=OUTWARD):
    a = np.array(x, np.float64); b = np.array(y, np.float64); r = np.zeros(2)
    lib().orc_iv_add(_dp(a), _dp(b), mode, _dp(r))
    return float(r[0]), float(r[1])


def iv_mul(x, y, mode=OUTWARD):
    a = np.array(x, np.float64); b = np.array(y, np.float64); r = np.zeros(2)
    lib().orc_iv_mul(_dp(a), _dp(b), mode, _dp(r))
    return float(r[0]), float(r[1])


def iv_muladd(x, y, c, mode=OUTWARD):
    """The Horner step x*y + c as one interval operation (each endpoint of the
    exact range rounded outward once); NEAREST: plain x*y, then + c."""
    a = np.array(x, np.float64); b = np.array(y, np.float64); d = np.array(c, np.float64); r = np.zeros(2)
    lib().orc_iv_muladd(_dp(a), _dp(b), _dp(d), mode, _dp(r))
    return float(r[0]), float(r[1])


def box(dlo: float, dhi: float, level: int, label: int):
    r = np.zeros(2)
    lib().orc_box(dlo, dhi, level, label, _dp(r))
    return float(r[0]), float(r[1])


def box_table(dlo: float, dhi: float, level: int, n: int | None = None) -> np.ndarray:
    """(n, 2) enclosures of the cells 0..n-1 of the 2^level grid on [dlo, dhi]."""
    n = (1 << level) if n is None else n
    out = np.zeros((n, 2))
    lib().orc_box_table(dlo, dhi, level, n, _dp(out))
    return out


# ---------------------------------------------------------------------------
# Evaluation
# ---------------------------------------------------------------------------

def _coef(poly):
    """(clo, chi, k, cube) from a cube or a (lo_cube, hi_cube) pair."""
    if isinstance(poly, tuple):
        lo = np.ascontiguousarray(poly[0], np.float64); hi = np.ascontiguousarray(poly[1], np.float64)
    else:
        lo = np.ascontiguousarray(poly, np.float64); hi = lo
    return lo, hi, lo.ndim, lo.shape[0]


def eval_box(poly, d: int, boxiv: np.ndarray, mode=OUTWARD):
    """Brute-force nested Horner on one box ((k,2) array). Returns (lo, hi, steps)."""
    lo, hi, k, cube = _coef(poly)
    b = np.ascontiguousarray(boxiv, np.float64).reshape(-1)
    r = np.zeros(2); st = C.c_int64(0)
    rc = lib().orc_eval_box(k, d, cube, _dp(lo), _dp(hi), _dp(b), mode, _dp(r), C.byref(st))
    if rc:
        raise ValueError("orc_eval_box failed")
    return float(r[0]), float(r[1]), int(st.value)


def eval_points(poly: np.ndarray, d: int, x: np.ndarray) -> np.ndarray:
    """Round-to-nearest point values by the same nested Horner order."""
    c = np.ascontiguousarray(poly, np.float64)
    k = c.ndim
    x = np.ascontiguousarray(x, np.float64).reshape(-1, k)
    f = np.zeros(x.shape[0])
    if lib().orc_eval_points(k, d, c.shape[0], _dp(c), _dp(x), x.shape[0], _dp(f)):
        raise ValueError("orc_eval_points failed")
    return f


def eval_csf(poly, d: int, csf: dict, tables: list, mode=OUTWARD, nthreads: int = 1):
    """Algorithm 2 on a box CSF.

    ``tables[l]`` is an (m_l, 2) array: the interval of each label on axis l.
    Returns (lo, hi, steps) with lo/hi in CSF leaf order and steps[l] the
    number of interval Horner steps spent at CSF depth l+1.
    """
    lo, hi, k, cube = _coef(poly)
    assert csf["k"] == k
    n = np.array([len(a) for a in csf["idx"]], np.int64)
    idx = [np.ascontiguousarray(a, np.int32) for a in csf["idx"]]
    ptr = [np.ascontiguousarray(a, np.int32) for a in csf["ptr"]] + [np.zeros(1, np.int32)] * (k - len(csf["ptr"]))
    tabs = [np.ascontiguousarray(t, np.float64) for t in tables]
    xn = np.array([t.shape[0] for t in tabs], np.int64)
    I32P = C.POINTER(C.c_int32)
    idx_arr = (I32P * k)(*[a.ctypes.data_as(I32P) for a in idx])
    ptr_arr = (I32P * k)(*[a.ctypes.data_as(I32P) for a in ptr])
    tab_arr = (C.POINTER(C.c_double) * k)(*[_dp(t) for t in tabs])
    nl = int(n[-1])
    olo = np.zeros(nl); ohi = np.zeros(nl); steps = np.zeros(k, np.int64)
    i64p = C.POINTER(C.c_int64)
    rc = lib().orc_eval_csf(k, d, cube, _dp(lo), _dp(hi), n.ctypes.data_as(i64p), idx_arr, ptr_arr,
                            tab_arr, xn.ctypes.data_as(i64p), mode, nthreads, _dp(olo), _dp(ohi),
                            steps.ctypes.data_as(i64p))
    if rc:
        raise ValueError("orc_eval_csf failed (bad arguments or labels outside the tables)")
    return olo, ohi, steps


# ---------------------------------------------------------------------------
# CSF of a set of grid indices (Sec. 2.1)
# ---------------------------------------------------------------------------

def csf_from_boxes(boxes: np.ndarray, level: int = 0) -> dict:
    """Canonical CSF of a set of index tuples (duplicates allowed, any order).

    Depth-l nodes are the distinct prefixes of length l+1, in lexicographic
    order; idx[l] holds their last coordinate and ptr[l][j] the position of
    the first child of node j among the depth-(l+1) nodes (ptr[l][-1] = N_{l+2}).
    """
    b = np.asarray(boxes, dtype=np.int64)
    k = b.shape[1]
    if b.shape[0]:
        b = np.unique(b, axis=0)  # lexicographic order of whole tuples
    idx, starts = [], []
    for l in range(k):
        if b.shape[0] == 0:
            flag = np.zeros(0, bool)
        else:
            flag = np.ones(b.shape[0], bool)
            flag[1:] = np.any(b[1:, : l + 1] != b[:-1, : l + 1], axis=1)
        st = np.flatnonzero(flag)
        starts.append(st)
        idx.append(b[st, l].astype(np.int32))
    ptr = []
    for l in range(k - 1):
        p = np.searchsorted(starts[l + 1], starts[l]).astype(np.int64)
        ptr.append(np.concatenate([p, [len(starts[l + 1])]]).astype(np.int32))
    return {"k": k, "level": level, "idx": idx, "ptr": ptr, "boxes": b.astype(np.int32)}


def csf_sizes(csf: dict) -> list:
    """N_1(S), ..., N_k(S) (Remark 1: number of nodes at each depth)."""
    return [len(a) for a in csf["idx"]]


def children_of(boxes: np.ndarray) -> np.ndarray:
    """All 2^k children 2*B + b of each box (bisection G_n -> G_2n, Sec. 3.2)."""
    b = np.asarray(boxes, np.int64)
    k = b.shape[1]
    bits = np.array(np.meshgrid(*([[0, 1]] * k), indexing="ij")).reshape(k, -1).T
    return (2 * b[:, None, :] + bits[None, :, :]).reshape(-1, k)


def level_tables(dom: np.ndarray, k: int, level: int) -> list:
    dom = np.asarray(dom, np.float64).reshape(k, 2)
    return [box_table(float(dom[j, 0]), float(dom[j, 1]), level) for j in range(k)]


def keep_mask(lo: np.ndarray, hi: np.ndarray) -> np.ndarray:
    """C0 over a system: keep a box unless some polynomial's enclosure excludes 0.

    lo/hi are (npolys, n).  A NaN endpoint never excludes (the comparison is
    false), so undefined enclosures keep their box.
    """
    excl = np.any((lo > 0) | (hi < 0), axis=0)
    return ~excl


def poly_degree(poly) -> int:
    c = poly[0] if isinstance(poly, tuple) else poly
    return c.shape[0] - 1


def eval_level(polys, csf: dict, dom: np.ndarray, nthreads: int = 1, mode=OUTWARD, degrees=None):
    """Enclosures of every polynomial on every leaf of the level's CSF."""
    k = csf["k"]
    tabs = level_tables(dom, k, csf["level"])
    los, his, steps = [], [], []
    for j, p in enumerate(polys):
        d = poly_degree(p) if degrees is None else degrees[j]
        lo, hi, st = eval_csf(p, d, csf, tabs, mode, nthreads)
        los.append(lo); his.append(hi); steps.append(st)
    return np.array(los).reshape(len(polys), -1), np.array(his).reshape(len(polys), -1), np.array(steps)


def subdivide(polys, k: int, depth: int, dom=None, nthreads: int = 1, start_level: int = 0,
              start_boxes=None, degrees=None):
    """Algorithm 3 with C0 only, stopped after `depth` (levels start_level..depth).

    Returns one record per level: the CSF S_l, the enclosures, the keep mask,
    the kept boxes K_l and the step counts.  S_{l+1} is the set of children of
    K_l.
    """
    dom = np.array([-1.0, 1.0] * k) if dom is None else np.asarray(dom, np.float64)
    boxes = np.zeros((1, k), np.int64) if start_boxes is None else np.asarray(start_boxes)
    out = []
    for level in range(start_level, depth + 1):
        S = csf_from_boxes(boxes, level)
        lo, hi, steps = eval_level(polys, S, dom, nthreads, degrees=degrees)
        keep = keep_mask(lo, hi)
        K = S["boxes"][keep]
        out.append({"level": level, "S": S, "lo": lo, "hi": hi, "keep": keep, "kept": K, "steps": steps})
        if level < depth:
            boxes = children_of(K)
    return out


def theorem1_steps(k: int, d: int, sizes: list) -> list:
    """Steps at each CSF depth: (Nt_{k-l} - Nt_{k-l-1}) * N_{l+1}(S) for a dense
    total-degree simplex, where Nt_m = C(d+m, m) counts the trailing m-tuples."""
    nt = [math.comb(d + m, m) for m in range(k + 1)]
    return [(nt[k - l] - nt[k - l - 1]) * sizes[l] for l in range(k)]


def order_costs(boxes: np.ndarray, level: int, degrees: list, orders: list) -> list:
    """Theorem 1 (Sec. 1, "Main Result") under each order of the variables:
    the CSF of the boxes with their labels listed in that order (depth l
    holds axis order[l]), its node counts, and the steps of evaluating dense
    total-degree polynomials of the given degrees on it.  Returns a list of
    (order, sizes, steps)."""
    boxes = np.asarray(boxes).reshape(-1, len(orders[0]))
    k = boxes.shape[1]
    out = []
    for o in orders:
        sizes = csf_sizes(csf_from_boxes(boxes[:, list(o)], level)) if len(boxes) else [0] * k
        out.append((tuple(o), sizes, sum(sum(theorem1_steps(k, d, sizes)) for d in degrees)))
    return out


# ---------------------------------------------------------------------------
# Mean-value exclusion (order-1 Taylor form, Sec. 3.2)
# ---------------------------------------------------------------------------

def centre_table(dlo: float, dhi: float, level: int, n: int | None = None) -> np.ndarray:
    """(n, 2) enclosures of the centres of cells 0..n-1 of the 2^level grid."""
    n = (1 << level) if n is None else n
    out = np.zeros((n, 2))
    lib().orc_centre_table(dlo, dhi, level, n, _dp(out))
    return out


def deriv(poly, d: int, axis: int):
    """Outward-rounded coefficient cubes (lo, hi) of dF/dx_axis (same side)."""
    lo, hi, k, cube = _coef(poly)
    olo = np.zeros_like(lo); ohi = np.zeros_like(lo)
    if lib().orc_deriv(k, d, cube, _dp(lo), _dp(hi), axis, _dp(olo), _dp(ohi)):
        raise ValueError("orc_deriv failed")
    return olo, ohi


def mean_value_level(polys, csf: dict, dom: np.ndarray, nthreads: int = 1, degrees=None):
    """Mean-value enclosures (lo, hi: (npolys, n)) on every leaf of the CSF:
    F(c) at the centre enclosures, each dF/dx_i on the boxes (Algorithm 2 on
    the same CSF), combined by ``orc_mean_value``."""
    k, level = csf["k"], csf["level"]
    dom = np.asarray(dom, np.float64).reshape(k, 2)
    btabs = level_tables(dom, k, level)
    ctabs = [centre_table(float(dom[j, 0]), float(dom[j, 1]), level) for j in range(k)]
    boxes = np.asarray(csf["boxes"], np.int64)
    nb = boxes.shape[0]
    bx = np.stack([btabs[j][boxes[:, j]] for j in range(k)], axis=1) if nb else np.zeros((0, k, 2))
    cx = np.stack([ctabs[j][boxes[:, j]] for j in range(k)], axis=1) if nb else np.zeros((0, k, 2))
    bx = np.ascontiguousarray(bx); cx = np.ascontiguousarray(cx)
    los, his = [], []
    for jp, p in enumerate(polys):
        d = poly_degree(p) if degrees is None else degrees[jp]
        fl, fh, _ = eval_csf(p, d, csf, ctabs, OUTWARD, nthreads)
        D = np.zeros((k, nb, 2))
        for i in range(k):
            if d == 0:
                continue
            dl, dh, _ = eval_csf(deriv(p, d, i), d - 1, csf, btabs, OUTWARD, nthreads)
            D[i, :, 0] = dl; D[i, :, 1] = dh
        fc = np.ascontiguousarray(np.stack([fl, fh], axis=1))
        out = np.zeros((nb, 2))
        if nb and lib().orc_mean_value(k, nb, _dp(fc), _dp(D), _dp(bx), _dp(cx), _dp(out)):
            raise ValueError("orc_mean_value failed")
        los.append(out[:, 0]); his.append(out[:, 1])
    return np.array(los).reshape(len(polys), -1), np.array(his).reshape(len(polys), -1)


def subdivide_mv(polys, k: int, depth: int, dom=None, nthreads: int = 1):
    """Algorithm 3 with the exclusion C0 and the mean-value test together: a
    box is dropped when, for some polynomial, either enclosure excludes 0."""
    dom = np.array([-1.0, 1.0] * k) if dom is None else np.asarray(dom, np.float64)
    boxes = np.zeros((1, k), np.int64)
    out = []
    for level in range(depth + 1):
        S = csf_from_boxes(boxes, level)
        lo, hi, steps = eval_level(polys, S, dom, nthreads)
        mlo, mhi = mean_value_level(polys, S, dom, nthreads)
        keep = keep_mask(lo, hi) & keep_mask(mlo, mhi)
        K = S["boxes"][keep]
        out.append({"level": level, "S": S, "lo": lo, "hi": hi, "mv_lo": mlo, "mv_hi": mhi, "keep": keep,
                    "kept": K})
        if level < depth:
            boxes = children_of(K)
    return out


# ---------------------------------------------------------------------------
# Order-2 Taylor form (Sec. 3.2, Taylor form definition with m = 2)
# ---------------------------------------------------------------------------

def taylor_pairs(k: int) -> list:
    """The pairs (i, j), i <= j, in lexicographic order (the order of the
    second-order terms and of the H_ij polynomials)."""
    return [(i, j) for i in range(k) for j in range(i, k)]


def deriv2(poly, d: int, i: int, j: int):
    """Outward-rounded coefficient cubes (lo, hi) of H_ij: (1/2) d2F/dx_i^2
    when i == j, d2F/dx_i dx_j when i < j (same side)."""
    lo, hi, k, cube = _coef(poly)
    olo = np.zeros_like(lo); ohi = np.zeros_like(lo)
    if lib().orc_deriv2(k, d, cube, _dp(lo), _dp(hi), i, j, _dp(olo), _dp(ohi)):
        raise ValueError("orc_deriv2 failed")
    return olo, ohi


def taylor2_level(polys, csf: dict, dom: np.ndarray, nthreads: int = 1, degrees=None):
    """Order-2 Taylor enclosures (lo, hi: (npolys, n)) on every leaf of the CSF:
    F(c) and every dF/dx_i(c) at the centre enclosures, every H_ij on the
    boxes (Algorithm 2 on the same CSF), combined by ``orc_taylor2``."""
    k, level = csf["k"], csf["level"]
    dom = np.asarray(dom, np.float64).reshape(k, 2)
    btabs = level_tables(dom, k, level)
    ctabs = [centre_table(float(dom[j, 0]), float(dom[j, 1]), level) for j in range(k)]
    boxes = np.asarray(csf["boxes"], np.int64)
    nb = boxes.shape[0]
    bx = np.stack([btabs[j][boxes[:, j]] for j in range(k)], axis=1) if nb else np.zeros((0, k, 2))
    cx = np.stack([ctabs[j][boxes[:, j]] for j in range(k)], axis=1) if nb else np.zeros((0, k, 2))
    bx = np.ascontiguousarray(bx); cx = np.ascontiguousarray(cx)
    los, his = [], []
    for jp, p in enumerate(polys):
        d = poly_degree(p) if degrees is None else degrees[jp]
        fc, D, H = _taylor2_parts(p, d, csf, btabs, ctabs, nthreads)
        out = np.zeros((nb, 2))
        if nb and lib().orc_taylor2(k, nb, _dp(fc), _dp(D), _dp(H), _dp(bx), _dp(cx), _dp(out)):
            raise ValueError("orc_taylor2 failed")
        los.append(out[:, 0]); his.append(out[:, 1])
    return np.array(los).reshape(len(polys), -1), np.array(his).reshape(len(polys), -1)


def _taylor2_parts(p, d, csf, btabs, ctabs, nthreads):
    """F and its first derivatives at the centre enclosures, the H_ij on the
    boxes: (fc (n, 2), D (k, n, 2), H (pairs, n, 2))."""
    k = csf["k"]
    nb = len(csf["boxes"])
    pairs = taylor_pairs(k)
    fl, fh, _ = eval_csf(p, d, csf, ctabs, OUTWARD, nthreads)
    D = np.zeros((k, nb, 2))
    for i in range(k):
        if d >= 1:
            dl, dh, _ = eval_csf(deriv(p, d, i), d - 1, csf, ctabs, OUTWARD, nthreads)
            D[i, :, 0] = dl; D[i, :, 1] = dh
    H = np.zeros((len(pairs), nb, 2))
    for t, (i, j) in enumerate(pairs):
        if d >= 2:
            hl, hh, _ = eval_csf(deriv2(p, d, i, j), d - 2, csf, btabs, OUTWARD, nthreads)
            H[t, :, 0] = hl; H[t, :, 1] = hh
    return np.ascontiguousarray(np.stack([fl, fh], axis=1)), D, H


def subdivide_t2(polys, k: int, depth: int, dom=None, nthreads: int = 1):
    """Algorithm 3 with the exclusion C0 and the order-2 Taylor test together:
    a box is dropped when, for some polynomial, either enclosure excludes 0."""
    dom = np.array([-1.0, 1.0] * k) if dom is None else np.asarray(dom, np.float64)
    boxes = np.zeros((1, k), np.int64)
    out = []
    for level in range(depth + 1):
        S = csf_from_boxes(boxes, level)
        lo, hi, steps = eval_level(polys, S, dom, nthreads)
        tlo, thi = taylor2_level(polys, S, dom, nthreads)
        keep = keep_mask(lo, hi) & keep_mask(tlo, thi)
        K = S["boxes"][keep]
        out.append({"level": level, "S": S, "lo": lo, "hi": hi, "t2_lo": tlo, "t2_hi": thi, "keep": keep,
                    "kept": K})
        if level < depth:
            boxes = children_of(K)
    return out


# ---------------------------------------------------------------------------
# Taylor form of any order m (Sec. 3.2, Taylor form definition)
# ---------------------------------------------------------------------------

def taylor_multi_indices(k: int, m: int) -> list:
    """The terms of the order-m form in the order they are summed: (j, alpha)
    for j = 0..m, the multi-indices of order j as the non-decreasing index
    tuples i_1 <= ... <= i_j in lexicographic order (j = 1: the axes; j = 2:
    the pairs of ``taylor_pairs``)."""
    out = []
    for j in range(m + 1):
        for tup in itertools.combinations_with_replacement(range(k), j):
            alpha = [0] * k
            for i in tup:
                alpha[i] += 1
            out.append((j, tuple(alpha)))
    return out


def taylor_coef(poly, d: int, alpha):
    """Outward-rounded coefficient cubes (lo, hi) of D^alpha F / alpha!: entry
    e is prod_i C(e_i + alpha_i, alpha_i) c_{e + alpha} (same side)."""
    lo, hi, k, cube = _coef(poly)
    a = (C.c_int32 * k)(*alpha)
    olo = np.zeros_like(lo); ohi = np.zeros_like(lo)
    rc = lib().orc_taylor_coef(k, d, cube, _dp(lo), _dp(hi), a, _dp(olo), _dp(ohi))
    if rc == -2:
        raise ValueError("Taylor coefficient multiplier reaches 2^53 (not exact in double)")
    if rc:
        raise ValueError("orc_taylor_coef failed")
    return olo, ohi


def taylor_m_level(polys, csf: dict, dom: np.ndarray, m: int, nthreads: int = 1, degrees=None):
    """Order-m Taylor enclosures (lo, hi: (npolys, n)) on every leaf of the
    CSF: the terms of orders 0..m-1 at the centre enclosures, those of order
    m on the boxes, every one by Algorithm 2 on the same CSF (a term whose
    order exceeds the degree is zero), combined by ``orc_taylor_m``."""
    k, level = csf["k"], csf["level"]
    dom = np.asarray(dom, np.float64).reshape(k, 2)
    btabs = level_tables(dom, k, level)
    ctabs = [centre_table(float(dom[j, 0]), float(dom[j, 1]), level) for j in range(k)]
    boxes = np.asarray(csf["boxes"], np.int64)
    nb = boxes.shape[0]
    bx = np.stack([btabs[j][boxes[:, j]] for j in range(k)], axis=1) if nb else np.zeros((0, k, 2))
    cx = np.stack([ctabs[j][boxes[:, j]] for j in range(k)], axis=1) if nb else np.zeros((0, k, 2))
    bx = np.ascontiguousarray(bx); cx = np.ascontiguousarray(cx)
    terms = taylor_multi_indices(k, m)
    alphas = np.ascontiguousarray(np.array([a for _, a in terms], np.int32).reshape(-1))
    los, his = [], []
    for jp, p in enumerate(polys):
        d = poly_degree(p) if degrees is None else degrees[jp]
        T = np.zeros((len(terms), nb, 2))
        for t, (j, alpha) in enumerate(terms):
            if j > d:
                continue
            coef = p if j == 0 else taylor_coef(p, d, alpha)
            tl, th, _ = eval_csf(coef, d - j, csf, btabs if j == m else ctabs, OUTWARD, nthreads)
            T[t, :, 0] = tl; T[t, :, 1] = th
        out = np.zeros((nb, 2))
        if nb and lib().orc_taylor_m(k, len(terms), alphas.ctypes.data_as(C.POINTER(C.c_int32)), nb,
                                     _dp(np.ascontiguousarray(T)), _dp(bx), _dp(cx), _dp(out)):
            raise ValueError("orc_taylor_m failed")
        los.append(out[:, 0]); his.append(out[:, 1])
    return np.array(los).reshape(len(polys), -1), np.array(his).reshape(len(polys), -1)


def subdivide_tm(polys, k: int, depth: int, m: int, dom=None, nthreads: int = 1):
    """Algorithm 3 with the exclusion C0 and the order-m Taylor test together:
    a box is dropped when, for some polynomial, either enclosure excludes 0."""
    dom = np.array([-1.0, 1.0] * k) if dom is None else np.asarray(dom, np.float64)
    boxes = np.zeros((1, k), np.int64)
    out = []
    for level in range(depth + 1):
        S = csf_from_boxes(boxes, level)
        lo, hi, steps = eval_level(polys, S, dom, nthreads)
        tlo, thi = taylor_m_level(polys, S, dom, m, nthreads)
        keep = keep_mask(lo, hi) & keep_mask(tlo, thi)
        K = S["boxes"][keep]
        out.append({"level": level, "S": S, "lo": lo, "hi": hi, "tm_lo": tlo, "tm_hi": thi, "keep": keep,
                    "kept": K})
        if level < depth:
            boxes = children_of(K)
    return out


# ---------------------------------------------------------------------------
# Inclusion criterion C1 (Sec. 3.2): sign change over the vertices of a box
# ---------------------------------------------------------------------------

def vertex_table(dlo: float, dhi: float, level: int, n: int | None = None) -> np.ndarray:
    """(n, 2) enclosures of the grid vertices 0..n-1 (n = 2^level + 1)."""
    n = (1 << level) + 1 if n is None else n
    out = np.zeros((n, 2))
    lib().orc_vertex_table(dlo, dhi, level, n, _dp(out))
    return out


def box_vertices(boxes: np.ndarray) -> np.ndarray:
    """(n, 2^k, k) vertex indices of each box: i + b for b in {0, 1}^k, b in
    binary order with the first axis most significant."""
    boxes = np.asarray(boxes, np.int64)
    n, k = boxes.shape
    bits = np.array([[(m >> (k - 1 - j)) & 1 for j in range(k)] for m in range(1 << k)], np.int64)
    return boxes[:, None, :] + bits[None, :, :]


def inclusion_level(polys, csf: dict, dom: np.ndarray, nthreads: int = 1, degrees=None):
    """C1 for every polynomial and box of the CSF: (np, n) booleans, true when
    some vertex's enclosure is > 0 and another's < 0 (so F vanishes in the box
    by the intermediate value theorem).  The vertices of all boxes form a set
    of grid points, evaluated once each by Algorithm 2 on its own CSF."""
    k, level = csf["k"], csf["level"]
    dom = np.asarray(dom, np.float64).reshape(k, 2)
    boxes = np.asarray(csf["boxes"], np.int64)
    nb = boxes.shape[0]
    out = np.zeros((len(polys), nb), bool)
    if nb == 0:
        return out
    vt = box_vertices(boxes).reshape(-1, k)
    V = csf_from_boxes(vt, level + 1)  # vertex labels run to 2^level
    vtabs = [vertex_table(float(dom[j, 0]), float(dom[j, 1]), level) for j in range(k)]
    keys = np.zeros(len(V["boxes"]), np.int64)
    q = np.zeros(len(vt), np.int64)
    for j in range(k):
        keys = keys * ((1 << level) + 1) + V["boxes"][:, j]
        q = q * ((1 << level) + 1) + vt[:, j]
    where = np.searchsorted(keys, q).reshape(nb, 1 << k)
    for jp, p in enumerate(polys):
        d = poly_degree(p) if degrees is None else degrees[jp]
        vl, vh, _ = eval_csf(p, d, V, vtabs, OUTWARD, nthreads)
        pos = (vl > 0.0)[where].any(axis=1)
        neg = (vh < 0.0)[where].any(axis=1)
        out[jp] = pos & neg
    return out


def taylor_inclusion_level(polys, csf: dict, dom: np.ndarray, nthreads: int = 1, degrees=None):
    """The Taylor-based C1 (Sec. 3.2, from the order-2 form) for every
    polynomial and box: (np, n) booleans, true when the order-2 bound of F at
    the vertex maximizing the linear part is > 0 and at the one minimizing it
    is < 0 (``orc_taylor_inclusion``)."""
    k, level = csf["k"], csf["level"]
    dom = np.asarray(dom, np.float64).reshape(k, 2)
    btabs = level_tables(dom, k, level)
    ctabs = [centre_table(float(dom[j, 0]), float(dom[j, 1]), level) for j in range(k)]
    vtabs = [vertex_table(float(dom[j, 0]), float(dom[j, 1]), level) for j in range(k)]
    boxes = np.asarray(csf["boxes"], np.int64)
    nb = boxes.shape[0]
    out = np.zeros((len(polys), nb), bool)
    if nb == 0:
        return out
    cx = np.ascontiguousarray(np.stack([ctabs[j][boxes[:, j]] for j in range(k)], axis=1))
    vl = np.ascontiguousarray(np.stack([vtabs[j][boxes[:, j]] for j in range(k)], axis=1))
    vu = np.ascontiguousarray(np.stack([vtabs[j][boxes[:, j] + 1] for j in range(k)], axis=1))
    for jp, p in enumerate(polys):
        d = poly_degree(p) if degrees is None else degrees[jp]
        fc, D, H = _taylor2_parts(p, d, csf, btabs, ctabs, nthreads)
        flags = np.zeros(nb, np.uint8)
        if lib().orc_taylor_inclusion(k, nb, _dp(fc), _dp(D), _dp(H), _dp(vl), _dp(vu), _dp(cx), flags):
            raise ValueError("orc_taylor_inclusion failed")
        out[jp] = flags.astype(bool)
    return out


def subdivide_c1(polys, k: int, depth: int, c1_from: int, dom=None, nthreads: int = 1, taylor: bool = False):
    """Algorithm 3 with both criteria: at every level the boxes excluded by C0
    are dropped; from level ``c1_from`` on (boxes smaller than the threshold)
    the kept boxes that satisfy C1 join the output R and are not bisected;
    the rest are bisected.  C1 is the vertex-sign test (or its Taylor form)
    for one polynomial and the Newton test for a system of 2..k polynomials
    (on the span of the gradients when there are fewer than k).  Per level:
    S, the C0 flags, the certified boxes and the continuing ones."""
    newton = 2 <= len(polys) <= k
    assert len(polys) == 1 or (newton and not taylor), "one polynomial, or a system of at most k"
    dom = np.array([-1.0, 1.0] * k) if dom is None else np.asarray(dom, np.float64)
    boxes = np.zeros((1, k), np.int64)
    out = []
    for level in range(depth + 1):
        S = csf_from_boxes(boxes, level)
        lo, hi, _ = eval_level(polys, S, dom, nthreads)
        keep = keep_mask(lo, hi)
        incl = np.zeros(len(keep), bool)
        if level >= c1_from and len(keep):
            if newton:
                fn = newton_level if len(polys) == k else newton_span_level
                incl = fn(polys, S, dom, nthreads)
            else:
                fn = taylor_inclusion_level if taylor else inclusion_level
                incl = fn(polys, S, dom, nthreads)[0]
        cert = keep & incl
        cont = keep & ~incl
        out.append({"level": level, "S": S, "keep": keep, "certified": S["boxes"][cert],
                    "kept": S["boxes"][cont]})
        if level < depth:
            boxes = children_of(S["boxes"][cont])
    return out


def slope_tables(dom: np.ndarray, k: int, level: int, j: int) -> list:
    """Axis tables of the slope column j: the cells on axes 0..j, the centre
    enclosures on axes j+1..k-1."""
    btabs = level_tables(dom, k, level)
    ctabs = [centre_table(float(dom[a, 0]), float(dom[a, 1]), level) for a in range(k)]
    return [btabs[a] if a <= j else ctabs[a] for a in range(k)]


def newton_level(polys, csf: dict, dom: np.ndarray, nthreads: int = 1, degrees=None, want_k: bool = False):
    """Newton interval test (Krawczyk's form) of a square system (k
    polynomials in k variables) on every leaf of the CSF: flags (n,) and,
    with ``want_k``, the enclosures K (n, k, 2).  F at the centre enclosures
    and the slopes S_ij = dF_i/dx_j on (B_1..B_j, c_{j+1}..c_k) come from
    Algorithm 2 on the same CSF; ``orc_krawczyk`` combines them."""
    k, level = csf["k"], csf["level"]
    assert len(polys) == k, "a square system"
    dom = np.asarray(dom, np.float64).reshape(k, 2)
    btabs = level_tables(dom, k, level)
    ctabs = [centre_table(float(dom[a, 0]), float(dom[a, 1]), level) for a in range(k)]
    vtabs = [vertex_table(float(dom[a, 0]), float(dom[a, 1]), level) for a in range(k)]
    boxes = np.asarray(csf["boxes"], np.int64)
    nb = boxes.shape[0]
    flags = np.zeros(nb, np.uint8)
    K = np.zeros((nb, k, 2))
    if nb == 0:
        return (flags.astype(bool), K) if want_k else flags.astype(bool)
    fc = np.zeros((k, nb, 2))
    Sm = np.zeros((k * k, nb, 2))
    for i, p in enumerate(polys):
        d = poly_degree(p) if degrees is None else degrees[i]
        fl, fh, _ = eval_csf(p, d, csf, ctabs, OUTWARD, nthreads)
        fc[i, :, 0] = fl; fc[i, :, 1] = fh
        for j in range(k):
            if d >= 1:
                sl, sh, _ = eval_csf(deriv(p, d, j), d - 1, csf, slope_tables(dom, k, level, j), OUTWARD, nthreads)
                Sm[i * k + j, :, 0] = sl; Sm[i * k + j, :, 1] = sh
    bx = np.ascontiguousarray(np.stack([btabs[a][boxes[:, a]] for a in range(k)], axis=1))
    cx = np.ascontiguousarray(np.stack([ctabs[a][boxes[:, a]] for a in range(k)], axis=1))
    inner = np.ascontiguousarray(np.stack([np.stack([vtabs[a][boxes[:, a], 1], vtabs[a][boxes[:, a] + 1, 0]], axis=1)
                                           for a in range(k)], axis=1))
    if lib().orc_krawczyk(k, nb, _dp(np.ascontiguousarray(fc)), _dp(np.ascontiguousarray(Sm)), _dp(bx), _dp(cx),
                          _dp(inner), flags, _dp(K)):
        raise ValueError("orc_krawczyk failed")
    return (flags.astype(bool), K) if want_k else flags.astype(bool)


def newton_span_level(polys, csf: dict, dom: np.ndarray, nthreads: int = 1, degrees=None, want_k: bool = False):
    """Newton test of a system of m < k polynomials on every leaf of the CSF
    (the square test on the span of the gradients at the box centre):
    flags (n,) and, with ``want_k``, the enclosures K (n, m, 2) in the
    plane's coordinates and the cube radii r (n,).  F and its first
    derivatives at the centre enclosures and the derivatives on the boxes
    come from Algorithm 2 on the same CSF; ``orc_newton_span`` combines them."""
    k, level = csf["k"], csf["level"]
    m = len(polys)
    assert 1 <= m < k, "fewer polynomials than variables"
    dom = np.asarray(dom, np.float64).reshape(k, 2)
    btabs = level_tables(dom, k, level)
    ctabs = [centre_table(float(dom[a, 0]), float(dom[a, 1]), level) for a in range(k)]
    boxes = np.asarray(csf["boxes"], np.int64)
    nb = boxes.shape[0]
    flags = np.zeros(nb, np.uint8)
    K = np.zeros((nb, m, 2))
    r = np.zeros(nb)
    if nb == 0:
        return (flags.astype(bool), K, r) if want_k else flags.astype(bool)
    fc = np.zeros((m, nb, 2))
    gc = np.zeros((m * k, nb, 2))
    D = np.zeros((m * k, nb, 2))
    for i, p in enumerate(polys):
        d = poly_degree(p) if degrees is None else degrees[i]
        fl, fh, _ = eval_csf(p, d, csf, ctabs, OUTWARD, nthreads)
        fc[i, :, 0] = fl; fc[i, :, 1] = fh
        for j in range(k):
            if d >= 1:
                dc = deriv(p, d, j)
                gl, gh, _ = eval_csf(dc, d - 1, csf, ctabs, OUTWARD, nthreads)
                gc[i * k + j, :, 0] = gl; gc[i * k + j, :, 1] = gh
                bl, bh, _ = eval_csf(dc, d - 1, csf, btabs, OUTWARD, nthreads)
                D[i * k + j, :, 0] = bl; D[i * k + j, :, 1] = bh
    bx = np.ascontiguousarray(np.stack([btabs[a][boxes[:, a]] for a in range(k)], axis=1))
    cx = np.ascontiguousarray(np.stack([ctabs[a][boxes[:, a]] for a in range(k)], axis=1))
    if lib().orc_newton_span(k, m, nb, _dp(np.ascontiguousarray(fc)), _dp(np.ascontiguousarray(gc)),
                             _dp(np.ascontiguousarray(D)), _dp(bx), _dp(cx), flags, _dp(K), _dp(r)):
        raise ValueError("orc_newton_span failed")
    return (flags.astype(bool), K, r) if want_k else flags.astype(bool)
