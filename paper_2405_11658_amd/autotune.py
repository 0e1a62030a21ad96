"""Parameter autotuning (host logic over the C ABI; every step of the method
runs in the library).

``autotune(h, warm, batch)`` - for one resident graph - tries candidate
settings of the asynchronous sweep's wavefront cap (``async_waves``: how many
vertices are in flight), of the degree above which a vertex takes the
multi-workgroup hub path instead of one wavefront with an LDS table
(``hub_degree``: which degree buckets get which table) and of the number of
hub slices (``hub_slices``) on scratch copies of the handle's current graph
and membership.  Each candidate
is run ``reps`` times: a scratch handle applies ``warm`` (which sizes its
work buffers) and then ``batch`` (valid after it, as ``inputs.batch_stream``
draws them) with the given front-end; the second update's latency (median
over the repetitions) and modularity (mean) are kept.  The reference is the
library's default setting, measured the same way: a candidate qualifies when
its mean modularity is at least the reference's minus ``q_tol``, and the
fastest qualifying candidate is installed on ``h`` with leiden_set_params;
``h``'s graph and membership are not touched.  The hub slice counts tried
start at 64, the smallest count whose modularity stays within 1e-3 of the
serial oracle's on RMAT-22 when both start from the same state.

``tune_fleet(graphs)`` - for the fused many-graph engine - times every launch
variant (wavefronts per workgroup x LDS table slots) on scratch fleets of the
given graphs running static Leiden, checks that all variants return the same
memberships (the engine's sweeps are serial, so they must) and returns the
fastest variant (median of ``reps`` launches).
"""
from __future__ import annotations

import itertools

import numpy as np
import torch

from . import leiden as L

DEFAULT_WAVES = (1024, 2048, 4096)
DEFAULT_SLICES = (64, 128)
DEFAULT_HUBDEG = (128, 256, 512)


def _scratch(off, idx, w, C, params):
    s = L.leiden_create(off, idx, w, params)
    L.leiden_set_state(s, C)
    return s


def _measure(off, idx, w, C, params, warm, batch, mode, reps):
    ms, qs = [], []
    for _ in range(reps):
        s = _scratch(off, idx, w, C, params)
        L.leiden_update(s, warm, mode, want_q=False)
        _, q, st, _ = L.leiden_update(s, batch, mode)
        ms.append(st["ms_total"] - st["ms_apply"])
        qs.append(q)
        L.leiden_destroy(s)
    return float(np.median(ms)), float(np.mean(qs))


def autotune(h: L.Handle, warm, batch, mode: str = "df", waves=DEFAULT_WAVES, slices=DEFAULT_SLICES,
             hubdeg=DEFAULT_HUBDEG, q_tol: float = 5e-4, reps: int = 3, base: L.leiden_params | None = None):
    """Returns (chosen params, reference (ms, q), list of (async_waves,
    hub_slices, hub_degree, ms, q) per candidate)."""
    off, idx, w = L.leiden_get_graph(h)
    C = L.leiden_get_state(h)[0].clone()
    base = base or L.leiden_default_params()
    ref = _measure(off, idx, w, C, base, warm, batch, mode, reps)
    results = []
    for aw, ns, hd in itertools.product(waves, slices, hubdeg):
        p = L.leiden_params.from_buffer_copy(base)
        p.async_waves = aw
        p.hub_slices = ns
        p.hub_degree = hd
        ms, q = _measure(off, idx, w, C, p, warm, batch, mode, reps)
        results.append((aw, ns, hd, ms, q))
    ok = [r for r in results if r[4] >= ref[1] - q_tol]
    chosen = L.leiden_params.from_buffer_copy(base)
    if ok:
        aw, ns, hd, ms, _ = min(ok, key=lambda r: r[3])
        if ms < ref[0]:
            chosen.async_waves = aw
            chosen.hub_slices = ns
            chosen.hub_degree = hd
    L.leiden_set_params(h, chosen)
    return chosen, ref, results


def tune_fleet(graphs, reps: int = 3, params: L.leiden_params | None = None):
    """graphs: list of (off, idx, w).  Returns (best variant, list of
    (variant, waves, slots, median ms))."""
    out = []
    ref = None
    for v in range(L.FLEET_VARIANTS):
        times = []
        for _ in range(reps):
            fl = L.Fleet(graphs, params)
            fl.set_variant(v)
            res, ms = fl.run([(k, "static", None) for k in range(len(graphs))])
            times.append(ms)
            mem = [r[0].clone() for r in res]
            fl.close()
        if ref is None:
            ref = mem
        elif not all(torch.equal(a, b) for a, b in zip(ref, mem)):
            raise RuntimeError(f"fleet variant {v} returned other memberships than variant 0")
        wv, sl = L.fleet_variant_info(v)
        out.append((v, wv, sl, float(np.median(times))))
    best = min(out, key=lambda r: r[3])[0]
    return best, out
