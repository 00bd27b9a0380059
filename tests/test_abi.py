"""The C-ABI library loads and exports every function declared in
include/edt.h; host-only entry points validate their arguments.  No kernel
is launched here, so this runs without a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "edt.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(edt_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    import paper_2105_04419_amd as m
    if not os.path.exists(m.LIB_PATH):
        m_build = __import__("paper_2105_04419_amd.build", fromlist=["build"])
        m_build.build()
    return m.lib()


def test_header_declares_the_boundary():
    fns = declared_functions()
    for name in ("edt_create", "edt_global", "edt_update", "edt_query", "edt_read_dense",
                 "edt_clearance_fwd", "edt_clearance_bwd", "edt_destroy"):
        assert name in fns


def test_every_declared_symbol_is_exported(L):
    missing = [f for f in declared_functions() if not hasattr(L, f)]
    assert not missing, missing


def test_status_strings(L):
    assert L.edt_status_str(0) == b"EDT_OK"
    assert L.edt_status_str(-3) == b"EDT_ERR_CAPACITY"
    assert L.edt_status_str(7) == b"EDT_UNKNOWN"


def test_workspace_bytes_validates(L):
    import paper_2105_04419_amd as m
    ok = m.EdtConfig(64, 64, 32, 20, 0, 0)
    n = L.edt_workspace_bytes(ctypes.byref(ok))
    assert n > 256 * 512 * 4
    for bad in [m.EdtConfig(0, 64, 32, 20, 0, 0), m.EdtConfig(64, 64, 32, 0, 0, 0),
                m.EdtConfig(64, 64, 32, 256, 0, 0), m.EdtConfig(64, 64, 32, 20, -1, 0)]:
        assert L.edt_workspace_bytes(ctypes.byref(bad)) == -1
    assert L.edt_workspace_bytes(None) == -1
    # a smaller pool needs less workspace
    small = m.EdtConfig(1024, 1024, 128, 32, 1000, 1000)
    big = m.EdtConfig(1024, 1024, 128, 32, 0, 0)
    assert 0 < L.edt_workspace_bytes(ctypes.byref(small)) < L.edt_workspace_bytes(ctypes.byref(big))


def test_create_rejects_bad_arguments_without_touching_the_gpu(L):
    import paper_2105_04419_amd as m
    cfg = m.EdtConfig(64, 64, 32, 20, 0, 0)
    out = ctypes.c_void_p()
    assert L.edt_create(ctypes.byref(cfg), None, 1 << 30, None, ctypes.byref(out)) == -1
    assert L.edt_create(ctypes.byref(cfg), ctypes.c_void_p(256), 16, None, ctypes.byref(out)) == -3
    assert L.edt_create(ctypes.byref(cfg), ctypes.c_void_p(257), 1 << 30, None,
                        ctypes.byref(out)) == -1
    assert L.edt_destroy(None) == -1
    assert L.edt_global(None, None, None) == -1
    assert L.edt_update(None, None, None, 0, None) == -1
    assert L.edt_clearance_fwd(None, 4, 4, 4, 0.2, 1.0, None, 1, 1, None, None) == -1


def test_dense_context_validates_without_touching_the_gpu(L):
    # workspace sizes: about 21 bytes per voxel plus the marks and the dedupe
    # table; invalid extents, change capacities and arguments are refused
    n = L.edt_dense_ctx_bytes(64, 32, 16, 100)
    assert n >= 21 * 64 * 32 * 16
    assert L.edt_dense_ctx_bytes(64, 32, 16, 1000) > n
    assert L.edt_dense_ctx_bytes(0, 32, 16, 100) == -1
    assert L.edt_dense_ctx_bytes(46341, 1, 1, 100) == -1
    assert L.edt_dense_ctx_bytes(8, 8, 8, 0) == -1
    out = ctypes.c_void_p()
    assert L.edt_dense_ctx_create(8, 8, 8, 0, 16, None, 1 << 20, None, ctypes.byref(out)) == -1
    assert L.edt_dense_ctx_create(8, 8, 8, -1, 16, ctypes.c_void_p(256), 1 << 20, None,
                                  ctypes.byref(out)) == -1
    assert L.edt_dense_ctx_create(8, 8, 8, 0, 16, ctypes.c_void_p(257), 1 << 20, None,
                                  ctypes.byref(out)) == -1
    assert L.edt_dense_ctx_create(8, 8, 8, 0, 16, ctypes.c_void_p(256), 64, None,
                                  ctypes.byref(out)) == -3
    assert L.edt_dense_ctx_update(None, None, None, 1, None) == -1
    assert L.edt_dense_ctx_global(None, None, None) == -1
    assert L.edt_dense_ctx_field(None) is None
    assert L.edt_dense_ctx_get_error(None, None) == -1


def test_product_package_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_2105_04419_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "edt_oracle" not in text, f
