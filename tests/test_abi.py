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
