"""CPU checks of the C ABI: the library loads and exports every declared symbol; host-side
argument checks answer without touching a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "spingp.h")
LIB = os.path.join(ROOT, "paper_1610_08035_amd", "libspingp.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(spingp_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libspingp.so is not built: run __graft_entry__.build()")
    return ctypes.CDLL(LIB)


def test_header_declares_the_hot_path_calls():
    names = declared_functions()
    for n in ("spingp_assemble", "spingp_factor", "spingp_solve", "spingp_logml", "spingp_selinv",
              "spingp_logml_grad", "spingp_create", "spingp_destroy", "spingp_status", "spingp_strerror"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    for n in declared_functions():
        assert hasattr(lib, n), n


def test_host_side_errors_without_gpu(lib):
    lib.spingp_strerror.restype = ctypes.c_char_p
    assert lib.spingp_strerror(3) == b"time points decrease inside a series"
    # null output handle, null terms, bad sizes: rejected before any device call
    assert lib.spingp_create(None, None, 1, 10, 1, None) == 1
    h = ctypes.c_void_p()
    assert lib.spingp_create(ctypes.byref(h), None, 1, 10, 1, None) == 1
    assert lib.spingp_factor(None) == 1
    assert lib.spingp_logml_grad(None, None, None, None) == 1
    assert lib.spingp_state_dim(None) == -1


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    import paper_1610_08035_amd.spingp as b
    monkeypatch.setattr(b, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(b, "_lib", None)
    with pytest.raises(RuntimeError, match="missing"):
        b.load_library()


def test_noalloc_host_errors_without_gpu(lib):
    """The allocation-free call rejects bad arguments and sizes beyond its fixed workspace before
    any device call (the pointers below are never dereferenced)."""
    class Term(ctypes.Structure):
        _fields_ = [("kind", ctypes.c_int32), ("harmonics", ctypes.c_int32)]

    f = lib.spingp_logml_grad_noalloc
    f.argtypes = [ctypes.POINTER(Term), ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    p = ctypes.c_void_p(0x1000)
    m52 = (Term * 1)(Term(2, 0))
    assert f(None, 1, p, p, 100, p, p, p, None) == 1                     # no terms
    assert f(m52, 1, None, p, 100, p, p, p, None) == 1                   # null t
    assert f(m52, 1, p, p, 0, p, p, p, None) == 1                        # empty series
    two = (Term * 2)(Term(1, 0), Term(3, 3))
    assert f(two, 2, p, p, 100, p, p, p, None) == 1                      # one term only
    assert f((Term * 1)(Term(3, 3)), 1, p, p, 100, p, p, p, None) == 8   # not a Matern term
    assert f(m52, 1, p, p, 142337, p, p, p, None) == 8                   # beyond the fixed workspace
    assert f((Term * 1)(Term(5, 0)), 1, p, p, 90113, p, p, p, None) == 8
