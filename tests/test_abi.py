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
    assert lib.spingp_logml_grad(None, None, None) == 1
    assert lib.spingp_state_dim(None) == -1


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    import paper_1610_08035_amd.spingp as b
    monkeypatch.setattr(b, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(b, "_lib", None)
    with pytest.raises(RuntimeError, match="missing"):
        b.load_library()
