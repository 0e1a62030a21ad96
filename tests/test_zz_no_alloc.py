"""GPU: leiden_modularity_noalloc (Eq. 1 with the library's fixed scratch,
no allocation, result left on the device) against leiden_modularity, on two
calls in a row (the second on a smaller graph, so stale scratch from the
first would show), plus the size limit."""
import ctypes as ct

import numpy as np
import pytest
import torch

from paper_2405_11658_amd import inputs as gen
from paper_2405_11658_amd import leiden as L

from .gpu_common import say

pytestmark = pytest.mark.gpu


def _noalloc(g, C):
    lib = L.load()
    f = lib.leiden_modularity_noalloc
    f.restype = ct.c_int32
    f.argtypes = [ct.c_int64, ct.c_int64] + [ct.c_void_p] * 6
    off = torch.as_tensor(g.off, device="cuda")
    idx = torch.as_tensor(g.idx, device="cuda")
    w = torch.as_tensor(g.w, device="cuda")
    Cd = torch.as_tensor(np.ascontiguousarray(C, np.int32), device="cuda")
    q = torch.full((1,), -7.0, dtype=torch.float64, device="cuda")
    st = f(g.n, g.nnz, L._ptr(off).value, L._ptr(idx).value, L._ptr(w).value, L._ptr(Cd).value, q.data_ptr(),
           torch.cuda.current_stream().cuda_stream)
    assert st == L.OK
    return float(q.item())


def test_modularity_noalloc_matches_leiden_modularity():
    big = gen.rmat(16, 16, seed=3)
        # the second graph is smaller: any stale scratch from the first call would show
    small = gen.planted_partition(1024, 16, 0.15, 0.005, seed=4)
    for g in (big, small):
        rng = np.random.default_rng(g.n)
        for labels in (np.arange(g.n), rng.integers(0, max(1, g.n // 64), g.n)):
            q1 = _noalloc(g, labels)
            q0 = L.leiden_modularity(g.off, g.idx, g.w, labels)
            say("n", g.n, "noalloc", q1, "leiden_modularity", q0)
            assert abs(q1 - q0) <= 1e-9 * max(1.0, abs(q0))


def test_modularity_noalloc_limits():
    lib = L.load()
    lib.leiden_modularity_noalloc_max_vertices.restype = ct.c_int64
    nmax = lib.leiden_modularity_noalloc_max_vertices()
    assert nmax >= 4 * 1024 * 1024
    f = lib.leiden_modularity_noalloc
    f.restype = ct.c_int32
    f.argtypes = [ct.c_int64, ct.c_int64] + [ct.c_void_p] * 6
    q = torch.zeros(1, dtype=torch.float64, device="cuda")
    fake = q.data_ptr()
    assert f(nmax + 1, 0, fake, None, None, fake, q.data_ptr(), None) == L.EINVAL   # beyond the scratch
    e = gen.from_edges(8, [], [])
    assert _noalloc(e, np.arange(8)) == 0.0                                       # no edges: Q = 0
