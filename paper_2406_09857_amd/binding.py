"""Thin Python binding of libvoxcsf.so (ctypes; argument marshalling only).

Every computation runs in the library's HIP kernels; torch provides device
memory and the current stream.  Function names follow the C ABI
(include/voxcsf.h): ``interval_eval_level``, ``filter_subdivide``,
``run_subdivision``, ``csf_build``.

A box set is a :class:`CSF`: per depth l (0-based) an int32 label tensor
``idx[l]`` and, for l < k-1, an int32 offset tensor ``ptr[l]``, plus the
host-side node counts ``n``.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvoxcsf.so")
KMAX = 4

VX_OK, VX_EINVAL, VX_ECAPACITY, VX_EHIP, VX_EOVERFLOW, VX_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
(VX_WS_EVAL, VX_WS_FILTER, VX_WS_BUILD, VX_WS_GRAD, VX_WS_MEANVALUE, VX_WS_TAYLOR2, VX_WS_INCLUSION, VX_WS_NEWTON,
 VX_WS_ORDER) = range(9)
VX_RUN_MEAN_VALUE, VX_RUN_TAYLOR2, VX_RUN_NO_TIMES, VX_RUN_INCLUSION, VX_RUN_INCLUSION_TAYLOR = 1, 2, 4, 8, 16
VX_RUN_EARLY_EXIT = 32
VX_RUN_AUTO_ORDER = 64


class VxError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"voxcsf error {code}: {msg}")
        self.code = code


class vx_poly(C.Structure):
    _fields_ = [("k", C.c_int32), ("degree", C.c_int32), ("side", C.c_int32), ("reserved", C.c_int32),
                ("c_lo", C.c_void_p), ("c_hi", C.c_void_p)]


class vx_csf(C.Structure):
    _fields_ = [("k", C.c_int32), ("level", C.c_int32), ("n", C.c_int64 * KMAX), ("cap", C.c_int64 * KMAX),
                ("idx", C.c_void_p * KMAX), ("ptr", C.c_void_p * KMAX)]


class vx_level_stat(C.Structure):
    _fields_ = [("level", C.c_int32), ("axes", C.c_int32), ("n", C.c_int64 * KMAX),
                ("kept", C.c_int64 * KMAX), ("steps", C.c_int64), ("eval_ms", C.c_double),
                ("filter_ms", C.c_double), ("certified", C.c_int64)]


class vx_kernel_stat(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("launches", C.c_int64), ("ms", C.c_double), ("units", C.c_double)]


# The same record as a numpy structured type, for converting a whole array
# of records at once (field access through ctypes costs microseconds each).
LEVEL_STAT_DTYPE = np.dtype({
    "names": [f for f, _ in vx_level_stat._fields_],
    "formats": [np.int32, np.int32, (np.int64, KMAX), (np.int64, KMAX), np.int64, np.float64, np.float64, np.int64],
    "offsets": [getattr(vx_level_stat, f).offset for f, _ in vx_level_stat._fields_],
    "itemsize": C.sizeof(vx_level_stat)})

LEVEL_CB = C.CFUNCTYPE(C.c_int, C.c_void_p, C.c_int32, C.POINTER(vx_csf), C.c_void_p, C.c_void_p, C.c_void_p,
                       C.POINTER(vx_csf))

_lib = None


def lib():
    """Load libvoxcsf.so; fails loudly when it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2406_09857_amd.build` "
                               "(or __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.vx_last_error.restype = C.c_char_p
        L.vx_workspace_bytes.argtypes = [C.c_int32, C.POINTER(vx_poly), C.c_int32, C.POINTER(vx_csf), C.c_int64]
        L.vx_workspace_bytes.restype = C.c_size_t
        L.interval_eval_level.argtypes = [C.POINTER(vx_poly), C.c_int32, C.POINTER(vx_csf), C.POINTER(C.c_double),
                                          vp, vp, vp, vp, C.c_size_t, vp]
        L.interval_eval_level_noalloc.argtypes = [C.POINTER(vx_poly), C.c_int32, C.POINTER(vx_csf),
                                                  C.POINTER(C.c_double), vp, vp, vp, vp]
        L.filter_subdivide.argtypes = [C.POINTER(vx_csf), vp, C.POINTER(vx_csf), C.POINTER(vx_csf), vp, vp,
                                       C.c_size_t, vp]
        L.run_subdivision.argtypes = [C.POINTER(vx_poly), C.c_int32, C.POINTER(C.c_double), C.c_int32, vp,
                                      C.c_size_t, C.POINTER(C.c_size_t), C.POINTER(vx_level_stat), LEVEL_CB, vp, vp]
        L.run_subdivision_ex.argtypes = [C.POINTER(vx_poly), C.c_int32, C.POINTER(C.c_double), C.c_int32, C.c_int32,
                                         vp, C.c_size_t, C.POINTER(C.c_size_t), C.POINTER(vx_level_stat), LEVEL_CB,
                                         vp, vp]
        L.mean_value_exclusion.argtypes = [C.POINTER(vx_poly), C.c_int32, C.POINTER(vx_csf), C.POINTER(C.c_double),
                                           vp, vp, vp, vp, C.c_size_t, vp]
        L.taylor_exclusion.argtypes = [C.POINTER(vx_poly), C.c_int32, C.POINTER(vx_csf), C.POINTER(C.c_double),
                                       C.c_int32, vp, vp, vp, vp, C.c_size_t, vp]
        L.inclusion_test.argtypes = [C.POINTER(vx_poly), C.c_int32, C.POINTER(vx_csf), C.POINTER(C.c_double), vp, vp,
                                     C.c_size_t, vp]
        L.taylor_inclusion_test.argtypes = L.inclusion_test.argtypes
        L.newton_test.argtypes = [C.POINTER(vx_poly), C.c_int32, C.POINTER(vx_csf), C.POINTER(C.c_double), vp, vp, vp,
                                  C.c_size_t, vp]
        L.csf_build.argtypes = [C.c_int32, C.c_int32, vp, C.c_int64, C.POINTER(vx_csf), vp, C.c_size_t, vp]
        L.variable_order_costs.argtypes = [C.POINTER(vx_poly), C.c_int32, C.POINTER(vx_csf), C.c_int32, vp, vp, vp,
                                           vp, C.c_size_t, vp]
        L.vx_taylor_workspace_bytes.argtypes = [C.POINTER(vx_poly), C.c_int32, C.POINTER(vx_csf), C.c_int32]
        L.vx_taylor_workspace_bytes.restype = C.c_size_t
        L.vx_copy.argtypes = [vp, vp, C.c_size_t, C.c_int32, vp]
        L.vx_profile_end.argtypes = [C.POINTER(vx_kernel_stat), C.c_int32, C.POINTER(C.c_int32)]
        L.vx_profile_select.argtypes = [C.c_char_p]
        for f in ("interval_eval_level", "interval_eval_level_noalloc", "filter_subdivide", "run_subdivision",
                  "run_subdivision_ex", "csf_build",
                  "vx_copy", "vx_profile_begin", "vx_profile_end", "vx_profile_select", "mean_value_exclusion",
                  "taylor_exclusion", "inclusion_test", "taylor_inclusion_test", "newton_test"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def _check(rc: int):
    if rc != VX_OK:
        raise VxError(rc, lib().vx_last_error().decode())


_PDOUBLE = C.POINTER(C.c_double)


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _dev(device=None):
    return torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)


# ---------------------------------------------------------------------------
# Data holders
# ---------------------------------------------------------------------------

@dataclass
class Poly:
    """A polynomial as a dense coefficient cube on the device (float64)."""
    c_lo: torch.Tensor
    c_hi: torch.Tensor | None = None
    degree: int | None = None

    def __post_init__(self):
        self.c_lo = self.c_lo.contiguous()
        if self.c_hi is not None:
            self.c_hi = self.c_hi.contiguous()
        if self.degree is None:
            self.degree = self.c_lo.shape[0] - 1

    @property
    def k(self) -> int:
        return self.c_lo.dim()

    def struct(self) -> vx_poly:
        return vx_poly(self.k, self.degree, self.c_lo.shape[0], 0, self.c_lo.data_ptr(),
                       self.c_hi.data_ptr() if self.c_hi is not None else None)


def as_polys(polys, device=None) -> list:
    out = []
    for p in polys:
        if isinstance(p, Poly):
            out.append(p)
        elif isinstance(p, tuple):
            out.append(Poly(torch.as_tensor(p[0], dtype=torch.float64, device=_dev(device)),
                            torch.as_tensor(p[1], dtype=torch.float64, device=_dev(device))))
        else:
            out.append(Poly(torch.as_tensor(np.asarray(p), dtype=torch.float64, device=_dev(device))))
    return out


def _poly_array(polys):
    arr = (vx_poly * len(polys))(*[p.struct() for p in polys])
    return arr


@dataclass
class CSF:
    """A box set of the 2^level grid as a CSF tree on the device."""
    k: int
    level: int
    idx: list
    ptr: list
    n: list = field(default_factory=list)

    def struct(self) -> vx_csf:
        s = vx_csf()
        s.k = self.k
        s.level = self.level
        for l in range(self.k):
            s.n[l] = int(self.n[l])
            s.cap[l] = int(self.idx[l].numel())
            s.idx[l] = self.idx[l].data_ptr()
            if l + 1 < self.k:
                s.ptr[l] = self.ptr[l].data_ptr()
        return s

    @staticmethod
    def empty(k: int, level: int, cap: list, device=None) -> "CSF":
        dev = _dev(device)
        idx = [torch.empty(max(1, int(c)), dtype=torch.int32, device=dev) for c in cap]
        ptr = [torch.empty(max(1, int(c)) + 1, dtype=torch.int32, device=dev) for c in cap[:-1]]
        return CSF(k, level, idx, ptr, [0] * k)

    @staticmethod
    def from_arrays(k: int, level: int, idx: list, ptr: list, device=None) -> "CSF":
        dev = _dev(device)
        ti = [torch.as_tensor(np.asarray(a, np.int32), device=dev) for a in idx]
        tp = [torch.as_tensor(np.asarray(a, np.int32), device=dev) for a in ptr]
        return CSF(k, level, ti, tp, [len(a) for a in idx])

    def trimmed(self) -> "CSF":
        return CSF(self.k, self.level, [self.idx[l][: self.n[l]] for l in range(self.k)],
                   [self.ptr[l][: self.n[l] + 1] for l in range(self.k - 1)], list(self.n))

    def to_numpy(self) -> dict:
        return {"k": self.k, "level": self.level,
                "idx": [self.idx[l][: self.n[l]].cpu().numpy() for l in range(self.k)],
                "ptr": [self.ptr[l][: self.n[l] + 1].cpu().numpy() for l in range(self.k - 1)]}

    @property
    def nboxes(self) -> int:
        return int(self.n[self.k - 1])


def _ws(nbytes: int, device=None) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=_dev(device))


# ---------------------------------------------------------------------------
# Entry points
# ---------------------------------------------------------------------------

def workspace_bytes(which: int, polys=None, csf: CSF | None = None, n: int = 0) -> int:
    parr = _poly_array(polys) if polys else None
    s = csf.struct() if csf is not None else None
    return int(lib().vx_workspace_bytes(which, parr, len(polys) if polys else 0, C.byref(s) if s else None, n))


def interval_eval_level(polys, csf: CSF, dom, out=None, keep: bool = True, ws=None, stream=None):
    """Enclosures (lo, hi: (np, nboxes) float64) and keep flags (uint8) of a
    polynomial system on every box of the CSF, in CSF leaf order."""
    polys = as_polys(polys)
    dom = np.ascontiguousarray(np.asarray(dom, np.float64).reshape(-1))
    nb = csf.nboxes
    dev = csf.idx[0].device
    if out is None:
        lo = torch.empty((len(polys), nb), dtype=torch.float64, device=dev)
        hi = torch.empty((len(polys), nb), dtype=torch.float64, device=dev)
        kp = torch.empty(max(nb, 1), dtype=torch.uint8, device=dev) if keep else None
    else:
        lo, hi, kp = out
    parr = _poly_array(polys)
    s = csf.struct()
    need = int(lib().vx_workspace_bytes(VX_WS_EVAL, parr, len(polys), C.byref(s), 0))
    if need == 0:
        _check(VX_EINVAL)
    if ws is None or ws.numel() < need:
        ws = _ws(need, dev)
    _check(lib().interval_eval_level(parr, len(polys), C.byref(s), dom.ctypes.data_as(C.POINTER(C.c_double)),
                                     lo.data_ptr(), hi.data_ptr(), kp.data_ptr() if kp is not None else None,
                                     ws.data_ptr(), ws.numel(), _stream(stream)))
    return lo, hi, (kp[:nb] if kp is not None else None)


NOALLOC_SCRATCH_BYTES = 64 << 20


def interval_eval_level_noalloc(polys, csf: CSF, dom, out=None, keep: bool = True, stream=None):
    """interval_eval_level with the library's static per-GPU scratch instead
    of a workspace (the C call allocates nothing; levels needing more than
    64 MiB of scratch raise VxError with VX_ECAPACITY)."""
    polys = as_polys(polys)
    dom = np.ascontiguousarray(np.asarray(dom, np.float64).reshape(-1))
    nb = csf.nboxes
    dev = csf.idx[0].device
    if out is None:
        lo = torch.empty((len(polys), nb), dtype=torch.float64, device=dev)
        hi = torch.empty((len(polys), nb), dtype=torch.float64, device=dev)
        kp = torch.empty(max(nb, 1), dtype=torch.uint8, device=dev) if keep else None
    else:
        lo, hi, kp = out
    parr = _poly_array(polys)
    s = csf.struct()
    _check(lib().interval_eval_level_noalloc(parr, len(polys), C.byref(s),
                                             dom.ctypes.data_as(C.POINTER(C.c_double)), lo.data_ptr(),
                                             hi.data_ptr(), kp.data_ptr() if kp is not None else None,
                                             _stream(stream)))
    return lo, hi, (kp[:nb] if kp is not None else None)


def mean_value_exclusion(polys, csf: CSF, dom, keep: torch.Tensor | None = None, stream=None):
    """Mean-value (order-1 Taylor form) enclosures (lo, hi: (np, nboxes)) on
    every box; ``keep`` (uint8, nboxes), if given, is cleared in place where
    some enclosure excludes 0."""
    return taylor_exclusion(polys, csf, dom, 1, keep, stream)


TAYLOR_MAX_ORDER = 6


def taylor_exclusion(polys, csf: CSF, dom, order: int, keep: torch.Tensor | None = None, stream=None):
    """Taylor-form enclosures of order 1..TAYLOR_MAX_ORDER (lo, hi: (np,
    nboxes)) on every box; ``keep`` (uint8, nboxes), if given, is cleared in
    place where some enclosure excludes 0."""
    polys = as_polys(polys)
    dom = np.ascontiguousarray(np.asarray(dom, np.float64).reshape(-1))
    nb = csf.nboxes
    dev = csf.idx[0].device
    lo = torch.empty((len(polys), max(nb, 1)), dtype=torch.float64, device=dev)
    hi = torch.empty((len(polys), max(nb, 1)), dtype=torch.float64, device=dev)
    parr = _poly_array(polys)
    s = csf.struct()
    need = int(lib().vx_taylor_workspace_bytes(parr, len(polys), C.byref(s), order))
    if need == 0:
        raise VxError(VX_EINVAL, f"invalid Taylor test of order {order} (order outside 1..{TAYLOR_MAX_ORDER}, "
                                 "too many polynomials for orders 1 and 2, or inconsistent polynomials and CSF)")
    ws = _ws(need, dev)
    _check(lib().taylor_exclusion(parr, len(polys), C.byref(s), dom.ctypes.data_as(C.POINTER(C.c_double)), order,
                                  lo.data_ptr(), hi.data_ptr(), keep.data_ptr() if keep is not None else None,
                                  ws.data_ptr(), ws.numel(), _stream(stream)))
    return lo[:, :nb], hi[:, :nb]


def filter_subdivide(csf: CSF, keep: torch.Tensor, want_kept: bool = True, want_next: bool = True, ws=None,
                     stream=None):
    """(kept CSF, next CSF) with host counts filled (synchronizes)."""
    k = csf.k
    dev = csf.idx[0].device
    kept = CSF.empty(k, csf.level, [csf.n[l] for l in range(k)], dev) if want_kept else None
    nxt = CSF.empty(k, csf.level + 1, [csf.n[l] << (l + 1) for l in range(k)], dev) if want_next else None
    d_counts = torch.zeros(2 * k, dtype=torch.int64, device=dev)
    s = csf.struct()
    need = int(lib().vx_workspace_bytes(VX_WS_FILTER, None, 0, C.byref(s), 0))
    if ws is None or ws.numel() < need:
        ws = _ws(need, dev)
    ks = kept.struct() if kept else None
    ns = nxt.struct() if nxt else None
    _check(lib().filter_subdivide(C.byref(s), keep.data_ptr(), C.byref(ks) if ks else None,
                                  C.byref(ns) if ns else None, d_counts.data_ptr(), ws.data_ptr(), ws.numel(),
                                  _stream(stream)))
    counts = d_counts.cpu().tolist()
    if kept:
        kept.n = counts[:k]
    if nxt:
        nxt.n = counts[k:]
    return kept, nxt


def root_csf(k: int, device=None) -> CSF:
    """The level-0 box set {(0, ..., 0)}."""
    return CSF.from_arrays(k, 0, [[0]] * k, [[0, 1]] * (k - 1), device)


def inclusion_test(polys, csf: CSF, dom, stream=None, taylor: bool = False) -> torch.Tensor:
    """Inclusion criterion C1: (np, nboxes) uint8, 1 where the polynomial
    certainly vanishes in the box (vertex enclosures of both strict signs);
    ``taylor=True`` uses the order-2 Taylor variant (bounds at the two
    extreme vertices of the linear part)."""
    polys = as_polys(polys)
    dom = np.ascontiguousarray(np.asarray(dom, np.float64).reshape(-1))
    nb = csf.nboxes
    dev = csf.idx[0].device
    incl = torch.empty((len(polys), max(nb, 1)), dtype=torch.uint8, device=dev)
    parr = _poly_array(polys)
    s = csf.struct()
    need = int(lib().vx_workspace_bytes(VX_WS_TAYLOR2 if taylor else VX_WS_INCLUSION, parr, len(polys),
                                        C.byref(s), 0))
    if need == 0:
        _check(VX_EINVAL)
    ws = _ws(need, dev)
    fn = lib().taylor_inclusion_test if taylor else lib().inclusion_test
    _check(fn(parr, len(polys), C.byref(s), dom.ctypes.data_as(C.POINTER(C.c_double)), incl.data_ptr(),
              ws.data_ptr(), ws.numel(), _stream(stream)))
    return incl[:, :nb]


def newton_test(polys, csf: CSF, dom, want_k: bool = False, stream=None):
    """Newton interval test (Krawczyk's form) of a system of np <= k
    polynomials on every box (np < k: on the span of the gradients at the box
    centre): (nboxes,) uint8, 1 where the system certainly has a zero in the
    box; with ``want_k`` also the enclosures K (nboxes, np, 2)."""
    polys = as_polys(polys)
    dom = np.ascontiguousarray(np.asarray(dom, np.float64).reshape(-1))
    nb = csf.nboxes
    dev = csf.idx[0].device
    incl = torch.empty(max(nb, 1), dtype=torch.uint8, device=dev)
    kout = torch.empty((max(nb, 1), len(polys), 2), dtype=torch.float64, device=dev) if want_k else None
    parr = _poly_array(polys)
    s = csf.struct()
    need = int(lib().vx_workspace_bytes(VX_WS_NEWTON, parr, len(polys), C.byref(s), 0))
    if need == 0:
        _check(VX_EINVAL)
    ws = _ws(need, dev)
    _check(lib().newton_test(parr, len(polys), C.byref(s), dom.ctypes.data_as(C.POINTER(C.c_double)),
                             incl.data_ptr(), kout.data_ptr() if want_k else None, ws.data_ptr(), ws.numel(),
                             _stream(stream)))
    return (incl[:nb], kout[:nb]) if want_k else incl[:nb]


def variable_order_costs(polys, csf: CSF, orders=None, stream=None):
    """Theorem 1's cost of evaluating the boxes of ``csf`` under each order
    of the variables (default: all k! orders, lexicographic).  Returns a
    list of (order, node counts N_1..N_k, interval Horner steps), computed by
    the library (one CSF build per order on the device)."""
    import itertools
    k = csf.k
    orders = [tuple(o) for o in (orders if orders is not None else itertools.permutations(range(k)))]
    parr = _poly_array(as_polys(polys)) if polys is not None else None
    s = csf.struct()
    need = int(lib().vx_workspace_bytes(VX_WS_ORDER, None, 0, C.byref(s), 0))
    if need == 0:
        _check(VX_EINVAL)
    ws = _ws(need, csf.idx[0].device)
    oa = np.ascontiguousarray(np.array(orders, np.int32).reshape(len(orders), k))
    counts = np.zeros((len(orders), k), np.int64)
    steps = np.zeros(len(orders), np.int64)
    _check(lib().variable_order_costs(parr, len(polys) if polys is not None else 0, C.byref(s), len(orders),
                                      oa.ctypes.data, counts.ctypes.data,
                                      steps.ctypes.data if polys is not None else None,
                                      ws.data_ptr(), ws.numel(), _stream(stream)))
    return [(o, [int(x) for x in counts[i]], int(steps[i]) if polys is not None else None)
            for i, o in enumerate(orders)]


def permute_variables(polys, order):
    """The polynomials with their variables reordered: new variable l is old
    variable order[l] (the coefficient cubes transposed on the host; interval
    pairs keep their pairing).  Boxes found for the result map back by
    listing their labels in the inverse order."""
    out = []
    for p in polys:
        if isinstance(p, tuple):
            out.append(tuple(np.ascontiguousarray(np.transpose(np.asarray(c), order)) for c in p))
        else:
            out.append(np.ascontiguousarray(np.transpose(np.asarray(p), order)))
    return out


def run_subdivision(polys, dom, depth: int, record=None, ws_bytes: int | None = None, stream=None,
                    ws: torch.Tensor | None = None, want_kept: bool = True, mean_value: bool = False,
                    taylor2: bool = False, level_times: bool = True, inclusion: str | None = None,
                    inclusion_from: int = 0, early_exit: bool = False, early_exit_from: int = 0,
                    taylor_order: int = 0, auto_order: bool = False, auto_order_at: int = 0):
    """Algorithm 3 with C0 to `depth`.  Returns (stats, kept) where stats is a
    list of per-level dicts and kept the final level's kept CSF (host numpy).
    ``mean_value`` / ``taylor2`` add the Taylor test of order 1 / 2 to C0,
    ``taylor_order=m`` the one of order m (1..TAYLOR_MAX_ORDER);
    ``level_times=False`` records no per-level timing events (eval_ms and
    filter_ms are then 0).  ``inclusion`` ("vertices" or "taylor") runs
    Algorithm 3 with C1 from level ``inclusion_from`` on: certified boxes
    leave the loop (keep = 2 in ``record``, counted in "certified").
    ``early_exit`` (systems) evaluates each polynomial only on the boxes the
    earlier ones kept: the same kept sets, fewer steps; ``record`` then gets
    lo = hi = keep = None; ``early_exit_from`` keeps the levels below it plain
    (the compaction pays only on large levels).

    ``auto_order`` runs in the order of the variables that Theorem 1 finds
    cheapest on the kept set of a probe level (``auto_order_at``, default
    min(depth, 6)); every CSF then lists its labels in that order, given in
    each stats record as "axes" (CSF depth l holds variable axes[l]).

    ``record(level, S, lo, hi, keep, K)`` is called with device-side views
    (numpy copies) when given; it may return True to stop.
    """
    polys = as_polys(polys)
    k = polys[0].k
    dom = np.ascontiguousarray(np.asarray(dom, np.float64).reshape(-1))
    parr = _poly_array(polys)
    stats = (vx_level_stat * (depth + 1))()
    need = C.c_size_t(0)
    final = {}

    def _copy_csf(cs) -> dict:
        out = {"k": k, "level": cs.level, "idx": [], "ptr": []}
        for l in range(k):
            a = np.empty(cs.n[l], np.int32)
            if cs.n[l]:
                _check(lib().vx_copy(a.ctypes.data, cs.idx[l], a.nbytes, 0, _stream(stream)))
            out["idx"].append(a)
            if l + 1 < k:
                b = np.empty(cs.n[l] + 1, np.int32)
                _check(lib().vx_copy(b.ctypes.data, cs.ptr[l], b.nbytes, 0, _stream(stream)))
                out["ptr"].append(b)
        return out

    def _cb(user, level, S, lo, hi, keep, K):
        try:
            if level == depth:
                final["kept"] = _copy_csf(K.contents)
            if record is not None:
                Sd = _copy_csf(S.contents)
                nb = S.contents.n[k - 1]
                lo_h = np.empty((len(polys), nb)); hi_h = np.empty((len(polys), nb)); kp = np.empty(nb, np.uint8)
                if not lo:
                    lo_h = hi_h = kp = None
                elif nb:
                    _check(lib().vx_copy(lo_h.ctypes.data, lo, lo_h.nbytes, 0, _stream(stream)))
                    _check(lib().vx_copy(hi_h.ctypes.data, hi, hi_h.nbytes, 0, _stream(stream)))
                    _check(lib().vx_copy(kp.ctypes.data, keep, kp.nbytes, 0, _stream(stream)))
                stop = record(level, Sd, lo_h, hi_h, kp, _copy_csf(K.contents))
                return 1 if stop else 0
            return 0
        except Exception as e:  # never let an exception cross the C boundary
            final["error"] = e
            return 1

    cb = LEVEL_CB(_cb) if (record is not None or want_kept) else LEVEL_CB()
    flags = ((VX_RUN_MEAN_VALUE if mean_value else 0) | (VX_RUN_TAYLOR2 if taylor2 else 0)
             | (0 if level_times else VX_RUN_NO_TIMES) | (VX_RUN_EARLY_EXIT if early_exit else 0)
             | (int(taylor_order) << 8) | (VX_RUN_AUTO_ORDER if auto_order else 0))
    if auto_order_at:
        if not auto_order or not 0 < auto_order_at < 16:
            raise ValueError("auto_order_at needs auto_order and a level in 1..15")
        flags |= auto_order_at << 12
    if early_exit_from:
        if not early_exit or not 0 < early_exit_from < 64:
            raise ValueError("early_exit_from needs early_exit and a level in 1..63")
        flags |= early_exit_from << 24
    if inclusion is not None:
        if inclusion not in ("vertices", "taylor"):
            raise ValueError("inclusion is 'vertices' or 'taylor'")
        flags |= (VX_RUN_INCLUSION if inclusion == "vertices" else VX_RUN_INCLUSION_TAYLOR) | (inclusion_from << 16)
    size = ws_bytes if ws_bytes is not None else (ws.numel() if ws is not None else 4 << 30)
    for _ in range(8):
        if ws is None or ws.numel() < size:
            ws = _ws(size)
        rc = lib().run_subdivision_ex(parr, len(polys), C.cast(dom.__array_interface__["data"][0], _PDOUBLE), depth,
                                      flags,
                                      ws.data_ptr(), ws.numel(),
                                      C.byref(need), stats, cb, None, _stream(stream))
        if rc == VX_ECAPACITY and need.value > size:
            size = int(need.value * 1.25)
            ws = None
            continue
        _check(rc)
        break
    if "error" in final:
        raise final["error"]
    a = np.frombuffer(stats, dtype=LEVEL_STAT_DTYPE)
    lv, ax, n, kp = a["level"].tolist(), a["axes"].tolist(), a["n"][:, :k].tolist(), a["kept"][:, :k].tolist()
    steps, em, fm, ce = a["steps"].tolist(), a["eval_ms"].tolist(), a["filter_ms"].tolist(), a["certified"].tolist()
    out = [{"level": lv[i], "n": n[i], "kept": kp[i], "steps": steps[i], "eval_ms": em[i], "filter_ms": fm[i],
            "certified": ce[i], "axes": [(ax[i] >> (4 * l)) & 15 for l in range(k)]} for i in range(len(lv))]
    return out, final.get("kept")


def profile_begin(only: str | None = None):
    """Start per-kernel HIP-event timing inside the library (of the kernel
    named `only`, or of every kernel)."""
    L = lib()
    _check(L.vx_profile_select(only.encode() if only else None))
    _check(L.vx_profile_begin())


def profile_end() -> dict:
    """Stop timing; {kernel name: {launches, ms, units}} (waits for the events)."""
    arr = (vx_kernel_stat * 64)()
    cnt = C.c_int32(0)
    _check(lib().vx_profile_end(arr, 64, C.byref(cnt)))
    return {arr[i].name.decode(): {"launches": int(arr[i].launches), "ms": float(arr[i].ms),
                                   "units": float(arr[i].units)} for i in range(min(cnt.value, 64))}


def csf_build(boxes: torch.Tensor, level: int, stream=None) -> CSF:
    """CSF of an (n, k) int32 device tensor of grid indices (any order,
    duplicates merged).  Synchronizes to read the node counts."""
    boxes = boxes.to(torch.int32).contiguous()
    n, k = int(boxes.shape[0]), int(boxes.shape[1])
    dev = boxes.device
    out = CSF.empty(k, level, [max(n, 1)] * k, dev)
    s = out.struct()
    probe = vx_csf()
    probe.k = k
    need = int(lib().vx_workspace_bytes(VX_WS_BUILD, None, 0, C.byref(probe), n))
    ws = _ws(need, dev)
    _check(lib().csf_build(k, level, boxes.data_ptr() if n else None, n, C.byref(s), ws.data_ptr(), ws.numel(),
                           _stream(stream)))
    out.n = [int(s.n[l]) for l in range(k)]
    return out


# ---------------------------------------------------------------------------
# Point evaluation, adjoint, Newton projection
# ---------------------------------------------------------------------------

def _grad_lib():
    L = lib()
    if not getattr(L, "_grad_ready", False):
        vp = C.c_void_p
        L.eval_grad.argtypes = [C.POINTER(vx_poly), C.c_int32, vp, C.c_int64, vp, vp, vp, vp, vp,
                                C.POINTER(vx_csf), C.POINTER(C.c_double), vp, C.c_size_t, vp]
        L.eval_grad.restype = C.c_int
        L.csf_centres.argtypes = [C.POINTER(vx_csf), C.POINTER(C.c_double), vp, vp]
        L.csf_centres.restype = C.c_int
        L.newton_project.argtypes = [C.POINTER(vx_poly), C.c_int32, vp, C.c_int64, C.c_int32, vp, vp, C.c_size_t,
                                     vp]
        L.newton_project.restype = C.c_int
        L.newton_project_grid.argtypes = [C.POINTER(vx_poly), C.c_int32, vp, C.c_int64, C.c_int32, vp,
                                          C.POINTER(vx_csf), C.POINTER(C.c_double), vp, C.c_size_t, vp]
        L.newton_project_grid.restype = C.c_int
        L._grad_ready = True
    return L


def csf_centres(csf: CSF, dom, stream=None) -> torch.Tensor:
    """(n, k) float64 centres of the leaf cells of a CSF."""
    dom = np.ascontiguousarray(np.asarray(dom, np.float64).reshape(-1))
    x = torch.empty((max(csf.nboxes, 1), csf.k), dtype=torch.float64, device=csf.idx[0].device)
    s = csf.struct()
    _check(_grad_lib().csf_centres(C.byref(s), dom.ctypes.data_as(C.POINTER(C.c_double)), x.data_ptr(),
                                   _stream(stream)))
    return x[: csf.nboxes]


def eval_grad(polys, x: torch.Tensor | None, want_jac: bool = True, gbar: torch.Tensor | None = None,
              want_xbar: bool = False, want_dcoef: bool = False, grid: CSF | None = None, dom=None, stream=None):
    """Point values f (np, n), Jacobian (n, np, k), and with gbar (np, n) the
    adjoints xbar (n, k) and dcoef (np, side^k cubes; needs `grid`).

    With ``grid`` (and ``dom``) the points are the centres of the grid's
    leaves: f and the Jacobian come from the amortized evaluation on the
    grid; ``x`` may then be None, and if given must equal those centres bit
    for bit (the library checks it and raises otherwise)."""
    polys = as_polys(polys)
    k = polys[0].k
    if x is None:
        if grid is None:
            raise ValueError("eval_grad needs points or a grid")
        n = grid.nboxes
        dev = grid.idx[0].device
    else:
        x = x.to(torch.float64).contiguous()
        n = int(x.shape[0])
        dev = x.device
    npl = len(polys)
    f = torch.empty((npl, max(n, 1)), dtype=torch.float64, device=dev)
    jac = torch.empty((max(n, 1), npl, k), dtype=torch.float64, device=dev) if want_jac else None
    xbar = torch.empty((max(n, 1), k), dtype=torch.float64, device=dev) if want_xbar else None
    dcoef = None
    if want_dcoef:
        dcoef = torch.zeros((npl,) + tuple(polys[0].c_lo.shape), dtype=torch.float64, device=dev)
    if gbar is not None:
        gbar = gbar.to(torch.float64).contiguous()
    parr = _poly_array(polys)
    gs = grid.struct() if grid is not None else None
    need = int(_grad_lib().vx_workspace_bytes(VX_WS_GRAD, parr, npl, C.byref(gs) if gs else None, n))
    if need == 0:
        _check(VX_EINVAL)
    ws = _ws(need, dev)
    domarr = np.ascontiguousarray(np.asarray(dom, np.float64).reshape(-1)) if dom is not None else None
    _check(_grad_lib().eval_grad(parr, npl, x.data_ptr() if (n and x is not None) else None, n, f.data_ptr(),
                                 jac.data_ptr() if jac is not None else None,
                                 gbar.data_ptr() if gbar is not None else None,
                                 xbar.data_ptr() if xbar is not None else None,
                                 dcoef.data_ptr() if dcoef is not None else None,
                                 C.byref(gs) if gs else None,
                                 domarr.ctypes.data_as(C.POINTER(C.c_double)) if domarr is not None else None,
                                 ws.data_ptr(), ws.numel(), _stream(stream)))
    return (f[:, :n], jac[:n] if jac is not None else None, xbar[:n] if xbar is not None else None, dcoef)


def newton_project(polys, x: torch.Tensor, steps: int = 3, stream=None, grid=None):
    """`steps` minimum-norm Newton steps on every point (in place); returns
    (x, F at the final points).  ``grid`` = (csf, dom) when x holds the
    centres of csf's leaves (checked): the first evaluation then runs on the
    CSF grid (``newton_project_grid``)."""
    polys = as_polys(polys)
    n = int(x.shape[0])
    f = torch.empty((len(polys), max(n, 1)), dtype=torch.float64, device=x.device)
    parr = _poly_array(polys)
    L = _grad_lib()
    if grid is None:
        need = int(L.vx_workspace_bytes(VX_WS_GRAD, parr, len(polys), None, n))
        ws = _ws(need, x.device)
        _check(L.newton_project(parr, len(polys), x.data_ptr(), n, steps, f.data_ptr(), ws.data_ptr(), ws.numel(),
                                _stream(stream)))
        return x, f[:, :n]
    csf, dom = grid
    cs = csf.struct()
    domv = np.ascontiguousarray(np.asarray(dom, np.float64).reshape(-1))
    need = int(L.vx_workspace_bytes(VX_WS_GRAD, parr, len(polys), C.byref(cs), n))
    ws = _ws(need, x.device)
    _check(L.newton_project_grid(parr, len(polys), x.data_ptr(), n, steps, f.data_ptr(), C.byref(cs),
                                 domv.ctypes.data_as(C.POINTER(C.c_double)), ws.data_ptr(), ws.numel(),
                                 _stream(stream)))
    return x, f[:, :n]


class PolyEval(torch.autograd.Function):
    """F(x) for a polynomial system as a torch autograd function.

    ``PolyEval.apply(x, grid, *coefs)``: x (n, k) float64 points, ``grid``
    None or a pair (csf, dom) whose leaf centres the points are, coefs one
    dense cube per polynomial (point coefficients); returns (np, n).  With a
    grid the library checks that x equals those centres bit for bit, the
    forward is the amortized evaluation on the grid, and the backward
    provides dL/dcoef (the transposed amortized evaluation); dL/dx is the
    forward-mode Jacobian contracted with the incoming gradient either way.
    Without a grid no coefficient gradient is provided.
    """

    @staticmethod
    def forward(ctx, x, grid, *coefs):
        polys = [Poly(c.detach().to(torch.float64)) for c in coefs]
        csf, dom = grid if grid is not None else (None, None)
        f, _, _, _ = eval_grad(polys, x.detach(), want_jac=False, grid=csf, dom=dom)
        ctx.save_for_backward(x, *coefs)
        ctx.grid = grid
        return f

    @staticmethod
    def backward(ctx, gf):
        x, *coefs = ctx.saved_tensors
        polys = [Poly(c.detach().to(torch.float64)) for c in coefs]
        want_dc = any(ctx.needs_input_grad[2:]) and ctx.grid is not None
        grid, dom = ctx.grid if ctx.grid is not None else (None, None)
        _, _, xbar, dcoef = eval_grad(polys, x.detach(), want_jac=False, gbar=gf.contiguous(),
                                      want_xbar=ctx.needs_input_grad[0], want_dcoef=want_dc, grid=grid, dom=dom)
        gx = xbar if ctx.needs_input_grad[0] else None
        gcs = [dcoef[i] if (want_dc and ctx.needs_input_grad[2 + i]) else None for i in range(len(coefs))]
        return (gx, None, *gcs)


# ---------------------------------------------------------------------------
# Batched subdivision of many independent systems
# ---------------------------------------------------------------------------

class vx_batch_tune(C.Structure):
    _fields_ = [("r1", C.c_int32), ("groups", C.c_int32), ("grid", C.c_int32), ("reserved", C.c_int32)]


class vx_batch_stat(C.Structure):
    _fields_ = [("level", C.c_int32), ("reserved", C.c_int32), ("n", C.c_int64 * KMAX),
                ("kept", C.c_int64 * KMAX), ("steps", C.c_int64), ("steps_depth", C.c_int64 * KMAX)]


VX_BATCH_GRAPH = 1


def _batch_lib():
    L = lib()
    if not getattr(L, "_batch_ready", False):
        vp = C.c_void_p
        i64p = C.POINTER(C.c_int64)
        L.vx_batch_workspace_bytes.argtypes = [C.POINTER(vx_poly), C.c_int32, C.c_int32, i64p]
        L.vx_batch_workspace_bytes.restype = C.c_size_t
        L.vx_batch_create.argtypes = [C.POINTER(vx_poly), C.c_int32, C.POINTER(C.c_double), C.c_int32, i64p,
                                      C.POINTER(vx_batch_tune), C.c_int32, vp, C.c_size_t, vp, C.POINTER(vp)]
        L.vx_batch_run.argtypes = [vp, vp]
        L.vx_batch_result.argtypes = [vp, C.POINTER(vx_batch_stat), i64p, C.POINTER(vx_csf), vp, vp, vp,
                                      C.POINTER(vx_csf), vp]
        L.vx_batch_autotune.argtypes = [vp, C.POINTER(vx_batch_tune), C.c_int32, C.c_int32,
                                        C.POINTER(vx_batch_tune), C.POINTER(C.c_float), vp]
        L.vx_batch_destroy.argtypes = [vp]
        L.vx_batch_destroy.restype = None
        for f in ("vx_batch_create", "vx_batch_run", "vx_batch_result", "vx_batch_autotune"):
            getattr(L, f).restype = C.c_int
        L._batch_ready = True
    return L


def _system_poly(s):
    """One polynomial per system: a cube, a Poly, or a one-element list."""
    if isinstance(s, list):
        if len(s) != 1:
            raise ValueError("the batched path takes one polynomial per system")
        s = s[0]
    return as_polys([s])[0]


def batch_caps_guess(nsys: int, depth: int) -> list:
    """Starting node capacities of a batched trivariate run: exact at depths 0
    and 1 (systems, x1 cells), a surface-sized guess below."""
    c2 = max(nsys * (4 ** depth) // 8, 4096)
    return [nsys, nsys << depth, c2, 4 * c2]


class Batch:
    """A batched run of independent systems (``vx_batch_*``): create once,
    ``run()`` many times (a HIP graph replay when ``graph``), ``result()``."""

    def __init__(self, systems, dom, depth: int, cap=None, tune=None, graph: bool = True, stream=None):
        L = _batch_lib()
        self.polys = [_system_poly(s) for s in systems]
        self.nsys = len(self.polys)
        self.k = self.polys[0].k
        self.depth = depth
        self.dom = np.ascontiguousarray(np.asarray(dom, np.float64).reshape(-1))
        self._parr = _poly_array(self.polys)
        self.cap = [int(c) for c in (cap if cap is not None else batch_caps_guess(self.nsys, depth))]
        capa = (C.c_int64 * KMAX)(*(self.cap + [0] * (KMAX - len(self.cap))))
        need = int(L.vx_batch_workspace_bytes(self._parr, self.nsys, depth, capa))
        if need == 0:
            _check(VX_EINVAL)
        self.ws = _ws(need)
        tarr = None
        if tune is not None:
            tarr = (vx_batch_tune * (depth + 1))(*[vx_batch_tune(*t, 0) for t in tune])
        h = C.c_void_p()
        _check(L.vx_batch_create(self._parr, self.nsys, self.dom.ctypes.data_as(C.POINTER(C.c_double)), depth, capa,
                                 tarr, VX_BATCH_GRAPH if graph else 0, self.ws.data_ptr(), self.ws.numel(),
                                 _stream(stream), C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _batch_lib().vx_batch_destroy(self._h)
            self._h = None
        self.ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, stream=None):
        _check(_batch_lib().vx_batch_run(self._h, _stream(stream)))

    def autotune(self, candidates=None, reps: int = 2, stream=None):
        """Per-level fastest of the candidates [(r1, groups, grid), ...];
        returns (chosen configs, per-level ms)."""
        if candidates is None:
            candidates = [(r, g, grid) for r in (1, 4, 8) for g in (1, 2, 4, 8, 16) for grid in (2048, 8192)]
        ca = (vx_batch_tune * len(candidates))(*[vx_batch_tune(*c, 0) for c in candidates])
        ch = (vx_batch_tune * (self.depth + 1))()
        ms = (C.c_float * (self.depth + 1))()
        _check(_batch_lib().vx_batch_autotune(self._h, ca, len(candidates), reps, ch, ms, _stream(stream)))
        return [(c.r1, c.groups, c.grid) for c in ch], list(ms)

    def result(self, want_last: bool = True, want_kept: bool = True, stream=None) -> dict:
        """Waits; per-level counts, high-water marks, the last level's
        evaluated set with enclosures and keep flags, and its kept set
        (outputs sized from the counts of a first, counts-only call)."""
        L = _batch_lib()
        nl = self.depth + 1
        kk = self.k + 1
        stats = (vx_batch_stat * nl)()
        need = (C.c_int64 * KMAX)()
        rc = L.vx_batch_result(self._h, stats, need, None, None, None, None, None, _stream(stream))
        st = np.array([[list(r.n), list(r.kept)] for r in stats], dtype=np.int64).reshape(nl, 2, KMAX)
        out = {"stats": st, "steps": [int(r.steps) for r in stats],
               "steps_depth": np.array([list(r.steps_depth)[: self.k] for r in stats], dtype=np.int64),
               "need": list(need)[:kk], "rc": rc}
        if rc != VX_OK:
            out["error"] = lib().vx_last_error().decode()
            return out
        if not (want_last or want_kept):
            return out
        nS, nK = [int(v) for v in st[self.depth, 0, :kk]], [int(v) for v in st[self.depth, 1, :kk]]
        dev = _dev()
        last = CSF.empty(kk, self.depth, nS, dev) if want_last else None
        kept = CSF.empty(kk, self.depth, nK, dev) if want_kept else None
        nb = max(1, nS[self.k])
        lo = torch.empty(nb, dtype=torch.float64, device=dev) if want_last else None
        hi = torch.empty(nb, dtype=torch.float64, device=dev) if want_last else None
        kp = torch.empty(nb, dtype=torch.uint8, device=dev) if want_last else None
        ls = last.struct() if last else None
        ks = kept.struct() if kept else None
        _check(L.vx_batch_result(self._h, None, None, C.byref(ls) if ls else None,
                                 lo.data_ptr() if lo is not None else None, hi.data_ptr() if hi is not None else None,
                                 kp.data_ptr() if kp is not None else None, C.byref(ks) if ks else None,
                                 _stream(stream)))
        if last:
            last.n = [int(ls.n[l]) for l in range(kk)]
            out.update(last=last, lo=lo[: nS[self.k]], hi=hi[: nS[self.k]], keep=kp[: nS[self.k]])
        if kept:
            kept.n = [int(ks.n[l]) for l in range(kk)]
            out["kept"] = kept
        return out


def split_systems(csf_np: dict, nsys: int) -> list:
    """Per-system leaf boxes ((n, k) int64, lexicographic) of a batched CSF
    given as numpy arrays (``CSF.to_numpy()``), plus each system's leaf
    range in the batched leaf order."""
    idx, ptr = csf_np["idx"], csf_np["ptr"]
    kk = len(idx)
    # parent of every node at each depth
    owner = [np.arange(len(idx[0]))]
    for l in range(1, kk):
        owner.append(np.repeat(np.arange(len(idx[l - 1])), np.diff(ptr[l - 1])))
    cols = []
    node = np.arange(len(idx[kk - 1]))
    for l in range(kk - 1, 0, -1):
        cols.append(idx[l][node])
        node = owner[l][node]
    sys_of_leaf = idx[0][node]
    boxes = np.stack(cols[::-1], axis=1).astype(np.int64) if cols else np.zeros((len(node), 0), np.int64)
    out = []
    for s in range(nsys):
        sel = np.nonzero(sys_of_leaf == s)[0]
        out.append({"boxes": boxes[sel], "leaves": sel})
    return out


def run_subdivision_batch(systems, dom, depth: int, graph: bool = True, autotune: bool = False, cap=None,
                          stream=None, max_tries: int = 6):
    """Batched Algorithm 3 (C0) on independent systems.  Grows the node
    capacities and retries when a run outgrows them.  Returns (Batch, result)."""
    cap = list(cap) if cap is not None else None
    for _ in range(max_tries):
        b = Batch(systems, dom, depth, cap=cap, graph=graph, stream=stream)
        b.run(stream)
        r = b.result(stream=stream)
        if r["rc"] == VX_ECAPACITY:
            cap = [max(int(n), 2 * c) if n >= c else c for n, c in zip(r["need"], b.cap)]
            b.close()
            del b
            continue
        if r["rc"] != VX_OK:
            raise VxError(r["rc"], r.get("error", ""))
        if autotune:
            b.autotune(stream=stream)
            b.run(stream)
            r = b.result(stream=stream)
            if r["rc"] != VX_OK:
                raise VxError(r["rc"], r.get("error", ""))
        return b, r
    raise VxError(VX_ECAPACITY, "batched run still outgrows its capacities")
