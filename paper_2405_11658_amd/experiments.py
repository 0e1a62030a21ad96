"""Experiment drivers around the C ABI (host code only; every step of the
method runs in the library's kernels).

* ``batch_sweep``: ND / DS / DF against static Leiden across batch sizes
  (Sec. 5.1.4: batches of 1e-7 |E| to 1e-1 |E|, 80 % insertions), each mode
  starting from the same installed membership on the same graph and batch;
  reports the update latency, the fraction of vertices marked affected, the
  fraction of communities flagged changed and the modularity (the measurements
  behind the paper's comparison of the front-ends, Sec. 5.2).
* ``temporal_stream``: a synthetic stand-in for the paper's temporal graphs
  (Sec. 5.1.3, 5.1.4): the edges of a graph are put in a seeded random order,
  the first 90 % are loaded, and the rest arrive as consecutive insertion
  batches, each applied with each front-end.

* ``served``: a scaled form of the served batched workload (many resident
  graphs, uneven batches), run as plain per-graph calls, through
  ``leiden_update_many`` and through the server.

Run ``python -m paper_2405_11658_amd.experiments sweep|stream|serve [options]``;
each prints one JSON object per measurement.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import inputs as gen

MODES = ("nd", "ds", "df")


def _leiden():
    from . import leiden as L  # loads the HIP library; fails loudly without it
    return L


def _handle(L, g, params=None):
    return L.leiden_create(g.off, g.idx, g.w, params)


def batch_sweep(scale: int = 22, edge_factor: int = 16, fracs=(1e-7, 1e-6, 1e-5, 1e-4, 1e-3, 1e-2, 1e-1),
                reps: int = 1, seed: int = 1, out=sys.stdout):
    """One JSON line per (fraction, repetition, mode) plus one for static Leiden."""
    L = _leiden()
    g = gen.rmat(scale, edge_factor, seed=seed)
    base = _handle(L, g)
    C0, q0, st0 = L.leiden_static(base)
    C0 = C0.clone()
    static_ms = st0["ms_total"]
    print(json.dumps({"kind": "static", "graph": f"rmat{scale}_ef{edge_factor}", "entries": int(g.nnz),
                      "ms": static_ms, "q": q0, "communities": int(C0.max().item()) + 1}), file=out, flush=True)
    for fi, f in enumerate(fracs):
        B = gen.batch_count(g.nnz, f)
        for r in range(reps):
            b = gen.random_batch(g, B, seed=seed + 1000 * fi + r)
            db = L.make_batch(b.del_u, b.del_v, b.ins_u, b.ins_v, b.ins_w)
            for mode in MODES:
                h = _handle(L, g)
                L.leiden_set_state(h, C0)
                _, q, st, _ = L.leiden_update(h, db, mode)
                lat = st["ms_total"] - st["ms_apply"]
                print(json.dumps({"kind": "update", "mode": mode, "frac": f, "batch": B, "rep": r,
                                  "ms": lat, "ms_graph_update": st["ms_apply"],
                                  "speedup_vs_static": static_ms / lat if lat > 0 else None,
                                  "affected_frac": st["affected"] / g.n,
                                  "changed": st["changed"], "passes": st["passes"], "q": q}),
                      file=out, flush=True)
                del h


def temporal_stream(scale: int = 20, edge_factor: int = 16, batches: int = 100, frac: float = 1e-4,
                    seed: int = 1, out=sys.stdout):
    """Preload 90 % of a graph's edges in a seeded random order, then stream
    `batches` insertion batches of round(frac * |E_T|) edges each; every mode
    follows the same stream on its own handle.  Static Leiden on the final
    graph gives the reference modularity."""
    L = _leiden()
    gT = gen.rmat(scale, edge_factor, seed=seed)
    src = np.repeat(np.arange(gT.n, dtype=np.int64), np.diff(gT.off))
    dst = gT.idx.astype(np.int64)
    und = np.flatnonzero(src < dst)
    order = np.random.default_rng(seed + 17).permutation(len(und))
    und = und[order]
    n0 = int(round(0.9 * len(und)))
    B = gen.batch_count(gT.nnz, frac)
    need = min(batches * B, len(und) - n0)
    g0 = gen.from_edges(gT.n, src[und[:n0]], dst[und[:n0]])
    stream = [und[n0 + k * B: min(n0 + (k + 1) * B, n0 + need)] for k in range((need + B - 1) // B)]
    empty = np.zeros(0, np.int32)
    for mode in MODES:
        h = _handle(L, g0)
        L.leiden_static(h)
        lat, q = [], None
        for e in stream:
            db = L.make_batch(empty, empty, src[e].astype(np.int32), dst[e].astype(np.int32),
                              np.ones(len(e), np.float32))
            _, q, st, _ = L.leiden_update(h, db, mode)
            lat.append(st["ms_total"] - st["ms_apply"])
        print(json.dumps({"kind": "stream", "mode": mode, "batches": len(stream), "batch": B,
                          "ms_p50": float(np.percentile(lat, 50)), "ms_p99": float(np.percentile(lat, 99)),
                          "ms_mean": float(np.mean(lat)), "q_final": q}), file=out, flush=True)
        del h
    h = _handle(L, gen.from_edges(gT.n, src[und[:n0 + need]], dst[und[:n0 + need]]))
    _, q, st = L.leiden_static(h)
    print(json.dumps({"kind": "stream_static", "ms": st["ms_total"], "q": q}), file=out, flush=True)


def served(graphs: int = 64, nmin: float = 1e3, nmax: float = 1e6, requests: int = 256, slots: int = 8,
           seed: int = 1, out=sys.stdout):
    """A scaled form of the served batched workload: `graphs` resident dynamic
    graphs with vertex counts log-uniform in [nmin, nmax] (half R-MAT with edge
    factor 8, half planted partitions of 64-vertex blocks), and `requests` DF
    update requests, each on a uniformly chosen graph with a batch of
    log-uniform 1e2..1e6 updates (80 % insertions) capped at 5 % of that
    graph's edges; the requests of one graph apply in order.  The same
    requests run three ways on the GPU, each from the same installed
    memberships: one update after another on one stream (plain per-graph
    calls); leiden_update_many over waves of distinct graphs; the server with
    `slots` workers, all requests queued at once (continuous batching).  One
    JSON line per form: updates per second of wall time, request latency
    p50/p99 and the mean final modularity."""
    L = _leiden()
    import torch
    rng = np.random.default_rng(seed)
    gs = []
    for k in range(graphs):
        n = int(round(np.exp(rng.uniform(np.log(nmin), np.log(nmax)))))
        if k % 2 == 0:
            scale = max(1, int(np.ceil(np.log2(n))))
            gs.append(gen.rmat(scale, 8, seed=seed + k, n=n))
        else:
            n = max(128, n // 64 * 64)
            gs.append(gen.planted_partition(n, n // 64, 0.1, 2.0 / n, seed=seed + k, permute=True))
    owner = rng.integers(0, graphs, requests)
    per = np.bincount(owner, minlength=graphs)
    streams = {}
    for k in range(graphs):
        if per[k] == 0:
            continue
        und = gs[k].nnz // 2
        size = int(round(np.exp(rng.uniform(np.log(1e2), np.log(1e6)))))
        size = max(1, min(size, und // 20 // max(1, per[k])))
        streams[k] = [L.make_batch(b.del_u, b.del_v, b.ins_u, b.ins_v, b.ins_w)
                      for b in gen.batch_stream(gs[k], size, int(per[k]), seed=seed + 100 + k)]
    order = []
    nxt = np.zeros(graphs, np.int64)
    for r in range(requests):
        k = int(owner[r])
        order.append((k, streams[k][nxt[k]]))
        nxt[k] += 1
    total_updates = sum(int(b[0].numel() + b[2].numel()) for _, b in order)
    entries = sum(g.nnz for g in gs)
    print(json.dumps({"kind": "serve_setup", "graphs": graphs, "requests": requests, "entries": int(entries),
                      "updates": total_updates}), file=out, flush=True)

    base = []
    for g in gs:
        h = L.leiden_create(g.off, g.idx, g.w)
        C, _, _ = L.leiden_static(h, want_q=False)
        base.append(C.clone())
        del h

    def fresh():
        hs = [L.leiden_create(g.off, g.idx, g.w) for g in gs]
        for h, C in zip(hs, base):
            L.leiden_set_state(h, C)
        torch.cuda.synchronize()
        return hs

    def report(form, wall, lats, hs):
        qs = [L.leiden_modularity(*L.leiden_get_graph(h), L.leiden_get_state(h)[0]) for h in hs]
        print(json.dumps({"kind": "serve", "form": form, "wall_s": round(wall, 3),
                          "updates_per_s": total_updates / wall, "requests_per_s": requests / wall,
                          "latency_p50_ms": float(np.percentile(lats, 50)),
                          "latency_p99_ms": float(np.percentile(lats, 99)),
                          "q_mean": float(np.mean(qs))}), file=out, flush=True)

    # plain per-graph calls, one after another (latency: from the start, as if
    # all requests were queued at time 0)
    hs = fresh()
    t0 = time.perf_counter()
    lats = []
    for k, b in order:
        L.leiden_update(hs[k], b, "df")
        lats.append((time.perf_counter() - t0) * 1e3)
    wall = time.perf_counter() - t0
    report("sequential", wall, lats, hs)
    del hs

    # waves of distinct graphs through leiden_update_many
    hs = fresh()
    t0 = time.perf_counter()
    lats = []
    wave, seen = [], set()
    def flush():
        if wave:
            res = L.leiden_update_many([hs[k] for k, _ in wave], [b for _, b in wave], ["df"] * len(wave),
                                       max_parallel=slots)
            assert all(r[3] == 0 for r in res)
            lats.extend([(time.perf_counter() - t0) * 1e3] * len(wave))
            wave.clear()
            seen.clear()
    for k, b in order:
        if k in seen:
            flush()
        wave.append((k, b))
        seen.add(k)
    flush()
    wall = time.perf_counter() - t0
    report("update_many", wall, lats, hs)
    del hs

    # the server: every request queued at once
    hs = fresh()
    sv = L.Server(slots=slots)
    t0 = time.perf_counter()
    ids = [sv.submit(hs[k], b, "df") for k, b in order]
    lats = []
    for rid in ids:
        st, _, _, _, lat, _ = sv.wait(rid)
        assert st == 0
        lats.append(lat)
    wall = time.perf_counter() - t0
    sv.close()
    report("server", wall, lats, hs)


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("sweep")
    s.add_argument("--scale", type=int, default=22)
    s.add_argument("--edge-factor", type=int, default=16)
    s.add_argument("--fracs", type=float, nargs="+", default=[1e-7, 1e-6, 1e-5, 1e-4, 1e-3, 1e-2, 1e-1])
    s.add_argument("--reps", type=int, default=1)
    t = sub.add_parser("stream")
    t.add_argument("--scale", type=int, default=20)
    t.add_argument("--edge-factor", type=int, default=16)
    t.add_argument("--batches", type=int, default=100)
    t.add_argument("--frac", type=float, default=1e-4)
    v = sub.add_parser("serve")
    v.add_argument("--graphs", type=int, default=64)
    v.add_argument("--nmax", type=float, default=1e6)
    v.add_argument("--requests", type=int, default=256)
    v.add_argument("--slots", type=int, default=8)
    a = ap.parse_args(argv)
    t0 = time.time()
    if a.cmd == "sweep":
        batch_sweep(a.scale, a.edge_factor, tuple(a.fracs), a.reps)
    elif a.cmd == "stream":
        temporal_stream(a.scale, a.edge_factor, a.batches, a.frac)
    else:
        served(a.graphs, 1e3, a.nmax, a.requests, a.slots)
    print(json.dumps({"kind": "done", "seconds": round(time.time() - t0, 1)}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
