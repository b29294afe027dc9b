"""CPU checks of the C-ABI boundary: the library loads and exports every
entry point declared in include/corutv.h; host-only calls behave."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "corutv.h")
LIB = os.path.join(ROOT, "paper_1906_04572_amd", "libcorutv.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(corutv_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libcorutv.so is not built; run __graft_entry__.build()")
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = declared()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n


def test_strerror_and_workspace_formula(lib):
    lib.corutv_strerror.restype = ctypes.c_char_p
    assert lib.corutv_strerror(0) == b"ok"
    assert b"invalid" in lib.corutv_strerror(-1)
    f = lib.corutv_workspace_bytes
    f.restype = ctypes.c_uint64
    f.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
    big = f(20000, 15000, 100, 10, 1, 1)
    assert big > 20000 * 112 * 8  # at least the FP64 bases
    assert f(15000, 20000, 100, 10, 1, 1) == big  # orientation-independent
    assert f(100, 50, 40, 20, 0, 0) == 0  # l > min(m, n)
    assert f(100, 50, 0, 5, 0, 0) == 0    # k < 1
    assert f(1000, 900, 250, 10, 0, 0) == 0  # l > 256
    assert f(100, 50, 10, 2, 0, 7) == 0   # bad precision


def test_null_arguments_are_rejected(lib):
    lib.corutv_create.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    assert lib.corutv_create(None, None) == -1
    lib.corutv_destroy.argtypes = [ctypes.c_void_p]
    assert lib.corutv_destroy(None) == -1


def test_binding_refuses_to_run_without_the_library(tmp_path):
    """The product path has no CPU fallback: a copy of the binding with no
    libcorutv.so beside it fails at import with a message naming the build."""
    import shutil
    import subprocess
    import sys

    pkg = tmp_path / "paper_1906_04572_amd"
    pkg.mkdir()
    shutil.copy(os.path.join(ROOT, "paper_1906_04572_amd", "__init__.py"), pkg / "__init__.py")
    code = ("import sys; sys.path.insert(0, %r)\n"
            "try:\n    import paper_1906_04572_amd\nexcept ImportError as e:\n    print('refused:', e)\n"
            "else:\n    print('loaded')\n") % str(tmp_path)
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert "refused:" in out.stdout and "not built" in out.stdout, (out.stdout, out.stderr)
