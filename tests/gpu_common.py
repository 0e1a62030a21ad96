"""Shared helpers of the GPU parity tests (host-side marshalling only)."""
import sys

import numpy as np
import torch

import oracle
from paper_2405_11658_amd import inputs as gen
from paper_2405_11658_amd import leiden as L


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


def og(g):
    return oracle.as_graph(g.n, g.off, g.idx, g.w)


def to_np(t):
    return t.detach().cpu().numpy()


def ob(b):
    return oracle.Batch(b.del_u, b.del_v, b.ins_u, b.ins_v, b.ins_w)


def dev_batch(b):
    return L.make_batch(b.del_u, b.del_v, b.ins_u, b.ins_v, b.ins_w)


def canon_rows(off, idx, w):
    """CSR -> dict row -> sorted list of (col, weight)."""
    off, idx, w = np.asarray(off), np.asarray(idx), np.asarray(w)
    out = {}
    for r in range(len(off) - 1):
        a, b = int(off[r]), int(off[r + 1])
        order = np.argsort(idx[a:b], kind="stable")
        out[r] = list(zip(idx[a:b][order].tolist(), w[a:b][order].tolist()))
    return out


def sync_params(**kw):
    return L.leiden_default_params(sync_mode=1, **kw)
