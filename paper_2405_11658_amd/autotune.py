"""Parameter autotuning for a resident graph (host logic over the C ABI; every
step of the method runs in the library).

``autotune(h, batch)`` tries candidate settings of the asynchronous sweep's
wavefront cap (``async_waves``: how many vertices are in flight) and of the
number of hub slices (``hub_slices``) on scratch copies of the handle's current
graph and membership: each candidate applies two sample batches one after
the other (``warm``, which sizes the scratch handle's work buffers, then
``batch``, valid after it, as ``inputs.batch_stream`` draws them) with the
given front-end, and the second update's latency and modularity are kept.  The fastest candidate whose modularity is within
``q_tol`` of the best modularity seen is installed on ``h`` with
leiden_set_params; ``h``'s graph and membership are not touched.
"""
from __future__ import annotations

import itertools

from . import leiden as L

DEFAULT_WAVES = (512, 1024, 2048, 4096)
DEFAULT_SLICES = (16, 32, 64)


def _scratch(off, idx, w, C, params):
    s = L.leiden_create(off, idx, w, params)
    L.leiden_set_state(s, C)
    return s


def autotune(h: L.Handle, warm, batch, mode: str = "df", waves=DEFAULT_WAVES, slices=DEFAULT_SLICES,
             q_tol: float = 5e-4, base: L.leiden_params | None = None):
    """Returns (chosen params, list of (async_waves, hub_slices, ms, q) per candidate)."""
    off, idx, w = L.leiden_get_graph(h)
    C = L.leiden_get_state(h)[0].clone()
    base = base or L.leiden_default_params()
    results = []
    for aw, ns in itertools.product(waves, slices):
        p = L.leiden_params.from_buffer_copy(base)
        p.async_waves = aw
        p.hub_slices = ns
        s = _scratch(off, idx, w, C, p)
        L.leiden_update(s, warm, mode, want_q=False)
        _, q, st, _ = L.leiden_update(s, batch, mode)
        results.append((aw, ns, st["ms_total"] - st["ms_apply"], q))
        L.leiden_destroy(s)
    qbest = max(r[3] for r in results)
    ok = [r for r in results if r[3] >= qbest - q_tol]
    aw, ns, _, _ = min(ok, key=lambda r: r[2])
    chosen = L.leiden_params.from_buffer_copy(base)
    chosen.async_waves = aw
    chosen.hub_slices = ns
    L.leiden_set_params(h, chosen)
    return chosen, results
