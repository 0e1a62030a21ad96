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


def test_update_many_argument_checks_without_a_device():
    lib = ct.CDLL(LIB)
    f = lib.leiden_update_many
    f.restype = ct.c_int32
    P, i32 = ct.c_void_p, ct.c_int32
    f.argtypes = [P, P, P, i32, P, P, P, P, i32, P]
    assert f(None, None, None, 0, None, None, None, None, 0, None) == 0      # nothing to do
    assert f(None, None, None, -1, None, None, None, None, 0, None) == 1     # negative count
    assert f(None, None, None, 2, None, None, None, None, 0, None) == 1     # missing arrays
    fake = (ct.c_void_p * 2)(0x1000, 0x1000)                                 # the same handle twice
    modes = (ct.c_int32 * 2)(3, 3)
    batches = (ct.c_char * 256)()
    assert f(fake, batches, modes, 2, None, None, None, None, 0, None) == 1
    nulls = (ct.c_void_p * 2)(None, None)
    assert f(nulls, batches, modes, 2, None, None, None, None, 0, None) == 1
    assert f(fake, batches, modes, 1, None, None, None, None, 65, None) == 1  # too many workers


def test_server_argument_checks_without_a_device():
    lib = ct.CDLL(LIB)
    P = ct.c_void_p
    lib.leiden_server_create.restype = ct.c_int32
    lib.leiden_server_create.argtypes = [ct.c_int32, ct.c_int64, P]
    out = ct.c_void_p()
    assert lib.leiden_server_create(0, 0, ct.byref(out)) == 1     # no slots
    assert lib.leiden_server_create(65, 0, ct.byref(out)) == 1    # too many
    assert lib.leiden_server_create(2, -1, ct.byref(out)) == 1    # negative budget
    assert lib.leiden_server_create(2, 0, None) == 1
    for name, args in (("leiden_server_submit", (None, None, None, 3, None, None)),
                       ("leiden_server_wait", (None, 1, None, None, None, None, None)),
                       ("leiden_server_destroy", (None,))):
        f = getattr(lib, name)
        f.restype = ct.c_int32
        assert f(*args) == 1


def test_boundary_argument_checks_without_a_device():
    """Marking, the update-size estimate and the allocator are checked before
    any HIP call."""
    lib = ct.CDLL(LIB)
    P, i32, i64 = ct.c_void_p, ct.c_int32, ct.c_int64
    lib.leiden_mark_affected.restype = i32
    lib.leiden_mark_affected.argtypes = [P, P, i32, P, P, P, P]
    assert lib.leiden_mark_affected(None, None, 3, None, None, None, None) == 1
    lib.leiden_update_bytes.restype = i32
    lib.leiden_update_bytes.argtypes = [P, i64, i64, P]
    out = ct.c_int64()
    assert lib.leiden_update_bytes(None, 1, 1, ct.byref(out)) == 1
    from paper_2405_11658_amd import leiden as L
    half = L.leiden_allocator()          # alloc and release both NULL
    lib.leiden_create.restype = i32
    lib.leiden_create.argtypes = [i64, i64, P, P, P, P, P, P, P]
    h = ct.c_void_p()
    off = (ct.c_int64 * 2)(0, 0)
    assert lib.leiden_create(1, 0, ct.cast(off, P), None, None, None, ct.byref(half), None, ct.byref(h)) == 1
    assert lib.leiden_create(-1, 0, ct.cast(off, P), None, None, None, None, None, ct.byref(h)) == 1
