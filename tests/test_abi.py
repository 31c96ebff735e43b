"""The C-ABI library loads and exports every entry point of include/voxcsf.h
(no GPU needed: nothing here launches work)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "voxcsf.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?(?:int|size_t|char\s*\*|void)\s*\*?\s*([a-z_][a-z0-9_]*)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["csf_build", "interval_eval_level", "filter_subdivide", "run_subdivision",
                     "vx_last_error", "vx_workspace_bytes", "vx_copy"]:
        assert required in names, required


def test_library_loads_and_exports_every_declared_symbol():
    from paper_2406_09857_amd import binding
    lib_path = binding.LIB_PATH
    if not os.path.exists(lib_path):
        pytest.fail("libvoxcsf.so is not built (run __graft_entry__.build())")
    L = binding.lib()
    out = subprocess.run(["nm", "-D", "--defined-only", lib_path], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (\S+)", out))
    for name in declared_functions():
        assert name in exported, name
        assert hasattr(L, name)


def test_error_path_without_gpu_work():
    """Argument errors are reported before anything is enqueued."""
    import ctypes as C
    from paper_2406_09857_amd import binding as b
    L = b.lib()
    s = b.vx_csf()
    s.k = 7  # invalid
    rc = L.interval_eval_level(None, 0, C.byref(s), None, None, None, None, None, 0, None)
    assert rc == b.VX_EINVAL
    rc = L.filter_subdivide(C.byref(s), None, None, None, None, None, 0, None)
    assert rc == b.VX_EINVAL
    assert b"k=7" in L.vx_last_error()


def test_misaligned_workspace_is_rejected_before_any_work():
    """The workspace contract (256-byte aligned) is checked on the host."""
    import ctypes as C
    from paper_2406_09857_amd import binding as b
    L = b.lib()
    s = b.vx_csf()
    s.k = 1
    s.level = 0
    s.n[0] = 0
    s.cap[0] = 1
    s.idx[0] = 256  # never dereferenced: no boxes
    parr = (b.vx_poly * 1)()
    parr[0].k, parr[0].degree, parr[0].side = 1, 1, 2
    parr[0].c_lo = 4096  # a device address in a real call; never dereferenced here
    dom = (C.c_double * 2)(-1.0, 1.0)
    rc = L.interval_eval_level(parr, 1, C.byref(s), dom, None, None, None, C.c_void_p(4096 + 8), 1 << 20, None)
    assert rc == b.VX_EINVAL and b"aligned" in L.vx_last_error()


def test_taylor_arguments_are_checked_before_any_work():
    """Orders outside 1..6 and the exclusive Taylor run flags are VX_EINVAL;
    the workspace query gives 0 for them."""
    import ctypes as C
    from paper_2406_09857_amd import binding as b
    L = b.lib()
    s = b.vx_csf()
    s.k = 1
    s.level = 0
    s.n[0] = 0
    s.cap[0] = 1
    s.idx[0] = 256  # never dereferenced
    parr = (b.vx_poly * 1)()
    parr[0].k, parr[0].degree, parr[0].side = 1, 1, 2
    parr[0].c_lo = 4096  # never dereferenced
    dom = (C.c_double * 2)(-1.0, 1.0)
    for bad in (0, 7, -1):
        rc = L.taylor_exclusion(parr, 1, C.byref(s), dom, bad, None, None, None, C.c_void_p(4096), 1 << 20, None)
        assert rc == b.VX_EINVAL and f"order {bad}".encode() in L.vx_last_error()
        assert L.vx_taylor_workspace_bytes(parr, 1, C.byref(s), bad) == 0
    for good in range(1, 7):  # an empty level: valid, nothing to do
        assert L.vx_taylor_workspace_bytes(parr, 1, C.byref(s), good) > 0
        rc = L.taylor_exclusion(parr, 1, C.byref(s), dom, good, None, None, None, C.c_void_p(4096), 1 << 20, None)
        assert rc == b.VX_OK
    for flags in (b.VX_RUN_MEAN_VALUE | b.VX_RUN_TAYLOR2, b.VX_RUN_TAYLOR2 | (3 << 8), b.VX_RUN_MEAN_VALUE | (4 << 8)):
        rc = L.run_subdivision_ex(parr, 1, dom, 2, flags, C.c_void_p(4096), 1 << 20, None, None, b.LEVEL_CB(),
                                  None, None)
        assert rc == b.VX_EINVAL and b"exclusive" in L.vx_last_error()
    rc = L.run_subdivision_ex(parr, 1, dom, 2, 7 << 8, C.c_void_p(4096), 1 << 20, None, None, b.LEVEL_CB(),
                              None, None)
    assert rc == b.VX_EINVAL and b"order 7" in L.vx_last_error()
    assert b.workspace_bytes(b.VX_WS_TAYLOR2) == 0  # invalid arguments give 0


def test_inclusion_run_flags_are_checked_before_any_work():
    """C1 in the loop needs one polynomial, one inclusion form, and an
    inclusion flag for a threshold level; the early exit takes neither."""
    import ctypes as C
    from paper_2406_09857_amd import binding as b
    L = b.lib()
    parr = (b.vx_poly * 2)()
    for i in range(2):
        parr[i].k, parr[i].degree, parr[i].side = 1, 1, 2
        parr[i].c_lo = 4096  # never dereferenced
    dom = (C.c_double * 2)(-1.0, 1.0)

    def run(np_, flags):
        return L.run_subdivision_ex(parr, np_, dom, 2, flags, C.c_void_p(4096), 1 << 20, None, None, b.LEVEL_CB(),
                                    None, None)

    assert run(2, b.VX_RUN_INCLUSION) == b.VX_EINVAL and b"one polynomial" in L.vx_last_error()
    assert run(1, b.VX_RUN_INCLUSION | b.VX_RUN_INCLUSION_TAYLOR) == b.VX_EINVAL
    assert b"exclusive" in L.vx_last_error()
    assert run(1, 3 << 16) == b.VX_EINVAL and b"without an inclusion flag" in L.vx_last_error()
    assert run(1, b.VX_RUN_EARLY_EXIT | b.VX_RUN_INCLUSION) == b.VX_EINVAL
    assert b"does not combine" in L.vx_last_error()
    assert run(1, 128) == b.VX_EINVAL and b"unknown flags" in L.vx_last_error()
    assert run(1, 5 << 12) == b.VX_EINVAL and b"AUTO_ORDER_AT without" in L.vx_last_error()


def test_binding_fails_loudly_without_the_library(tmp_path, monkeypatch):
    """No CPU fallback: with the library missing, loading it (which every
    entry point of the binding does first) raises."""
    from paper_2406_09857_amd import binding as b
    monkeypatch.setattr(b, "_lib", None)
    monkeypatch.setattr(b, "LIB_PATH", str(tmp_path / "libvoxcsf.so"))
    with pytest.raises(RuntimeError, match="missing"):
        b.lib()


def test_variable_order_arguments_are_checked_before_any_work():
    """Orders that are not permutations of 0..k-1, and a count outside
    1..24, are VX_EINVAL before anything touches the device."""
    import ctypes as C
    from paper_2406_09857_amd import binding as b
    L = b.lib()
    s = b.vx_csf()
    s.k = 2
    s.level = 1
    for l in range(2):
        s.n[l] = 0
        s.cap[l] = 1
        s.idx[l] = 256  # never dereferenced
    s.ptr[0] = 512
    counts = (C.c_int64 * 8)()
    for bad in ((0, 0), (0, 2), (-1, 1)):
        o = (C.c_int32 * 2)(*bad)
        rc = L.variable_order_costs(None, 0, C.byref(s), 1, o, counts, None, C.c_void_p(4096), 1 << 20, None)
        assert rc == b.VX_EINVAL and b"permutation" in L.vx_last_error()
    o = (C.c_int32 * 2)(1, 0)
    assert L.variable_order_costs(None, 0, C.byref(s), 0, o, counts, None, C.c_void_p(4096), 1 << 20,
                                  None) == b.VX_EINVAL
    assert b.workspace_bytes(b.VX_WS_ORDER) == 0  # invalid arguments give 0


def test_bench_refuses_more_than_one_gpu():
    """bench.py runs on one GPU: --gpus 2 exits with status 2 and says why,
    before it imports torch or touches a device."""
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2", "--no-cpu-baseline"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr and not r.stdout.strip()


def test_next_level_bound_overflow_is_refused_before_any_work():
    """Bisection gives depth l + 1 up to 2^(l+1) n[l] nodes; labels and
    offsets are int32, so a level whose children could reach 2^31 - 1 at
    some depth is VX_EOVERFLOW (the same host check sizes the level loop's
    next level), and one just below the limit passes that check."""
    import ctypes as C
    from paper_2406_09857_amd import binding as b
    L = b.lib()

    def csf(n, level=20):
        s = b.vx_csf()
        s.k = 3
        s.level = level
        for l in range(3):
            s.n[l] = n[l]
            s.cap[l] = n[l]
            s.idx[l] = 256 * (l + 1)  # never dereferenced: the call fails first
        s.ptr[0], s.ptr[1] = 4096, 8192
        return s

    nxt = b.vx_csf()
    nxt.k = 3
    keep = C.c_void_p(1 << 20)
    S = csf([1 << 10, 1 << 20, 1 << 28])  # depth 3: 2^28 << 3 = 2^31
    rc = L.filter_subdivide(C.byref(S), keep, None, C.byref(nxt), None, None, 0, None)
    assert rc == b.VX_EOVERFLOW and b"int32" in L.vx_last_error()
    S = csf([1 << 29, 1 << 29, 1 << 29])  # depth 1: 2^29 << 1 = 2^30 fits; depth 2: 2^31 does not
    rc = L.filter_subdivide(C.byref(S), keep, None, C.byref(nxt), None, None, 0, None)
    assert rc == b.VX_EOVERFLOW and b"depth 2" in L.vx_last_error()
    # just below the limit: the bound check passes and the (empty) next CSF's capacity is what fails
    S = csf([1 << 10, 1 << 20, (1 << 28) - 1])
    rc = L.filter_subdivide(C.byref(S), keep, None, C.byref(nxt), None, None, 0, None)
    assert rc == b.VX_ECAPACITY and b"next CSF" in L.vx_last_error()
    # without a next CSF nothing is bisected, so no bound applies
    kept = b.vx_csf()
    kept.k = 3
    rc = L.filter_subdivide(C.byref(S), keep, C.byref(kept), None, None, None, 0, None)
    assert rc == b.VX_ECAPACITY and b"kept CSF" in L.vx_last_error()
    # level 29 cannot be bisected at all
    S = csf([1, 1, 1], level=29)
    rc = L.filter_subdivide(C.byref(S), keep, None, C.byref(nxt), None, None, 0, None)
    assert rc == b.VX_EOVERFLOW and b"level 29" in L.vx_last_error()
