"""CPU-only checks of the C ABI: the library loads and exports every entry
point declared in include/leiden.h; host-only helpers behave."""
import ctypes as ct
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "leiden.h")
LIB = os.path.join(ROOT, "paper_2405_11658_amd", "libleiden_hip.so")


def declared_functions():
    text = open(HDR).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(leiden_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("leiden_create", "leiden_static", "leiden_update", "leiden_modularity",
                     "leiden_aggregate", "leiden_destroy"):
        assert required in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "build the library first (paper_2405_11658_amd/build.py)"
    lib = ct.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_host_only_helpers():
    lib = ct.CDLL(LIB)
    from paper_2405_11658_amd import leiden as L
    p = L.leiden_params()
    lib.leiden_default_params(ct.byref(p))
    assert (p.tau0, p.tol_drop, p.agg_tol, p.max_iter, p.max_passes) == (0.01, 10.0, 1.0, 20, 10)
    lib.leiden_strerror.restype = ct.c_char_p
    assert lib.leiden_strerror(1) == b"invalid argument"
    assert lib.leiden_strerror(3).startswith(b"no community state")


def test_null_arguments_are_rejected_without_a_device():
    lib = ct.CDLL(LIB)
    lib.leiden_update.restype = ct.c_int32
    lib.leiden_destroy.restype = ct.c_int32
    # argument checks happen before any HIP call
    assert lib.leiden_update(None, None, 3, None, None, None, None, None) == 1
    assert lib.leiden_destroy(None) == 1


def test_binding_fails_loudly_without_library(monkeypatch):
    from paper_2405_11658_amd import leiden as L
    monkeypatch.setattr(L, "LIB_PATH", "/nonexistent/libleiden_hip.so")
    monkeypatch.setattr(L, "_lib", None)
    with pytest.raises(ImportError):
        L.load()
