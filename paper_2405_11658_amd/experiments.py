"""Experiment drivers around the C ABI (host code only; every step of the
method runs in the library's kernels).

* ``batch_sweep``: ND / DS / DF against static Leiden across batch sizes
  (Sec. 5.1.4: batches of 1e-7 |E| to 1e-1 |E|, 80 % insertions), each mode
  starting from the same installed membership on the same graph and batch;
  reports the update latency, the fraction of vertices marked affected, the
  fraction of communities flagged changed and the modularity (the measurements
  behind the paper's comparison of the front-ends, Sec. 5.2).
* ``temporal_stream``: the paper's temporal protocol (Sec. 5.1.3, 5.1.4) on a
  synthetic stand-in: the edges of a graph arrive in a seeded random order,
  the first 90 % are loaded, then 100 consecutive batches of 1e-5, 1e-4 and
  1e-3 |E_T| (80 % arrivals, 20 % deletions) are applied with each
  front-end.

* ``served``: the served batched workload (256 resident graphs of 1e3-1e7
  vertices, Poisson-arriving uneven batches): plain per-graph calls against
  the server (small graphs as fleet jobs gathered into persistent launches,
  large ones as handles) at saturation and at offered loads of 0.5, 0.8 and
  1.0 times the saturation rate.

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


def _inverse(L, b):
    """The batch that undoes b: its insertions deleted, its deletions
    inserted again (unit weights, as the generators draw)."""
    return L.make_batch(b.ins_u, b.ins_v, b.del_u, b.del_v, np.ones(len(b.del_u), np.float32))


def _warm(L, h, C0, b, db, mode):
    """Sizes h's work buffers for this graph and batch (the batch, then its
    inverse), and installs C0 again: the next update of db is measured
    without first-call allocations, on the same graph."""
    L.leiden_update(h, db, mode, want_q=False)
    L.leiden_update(h, _inverse(L, b), mode, want_q=False)
    L.leiden_set_state(h, C0)


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
                _warm(L, h, C0, b, db, mode)
                _, q, st, _ = L.leiden_update(h, db, mode)
                lat = st["ms_total"] - st["ms_apply"]
                print(json.dumps({"kind": "update", "mode": mode, "frac": f, "batch": B, "rep": r,
                                  "ms": lat, "ms_graph_update": st["ms_apply"],
                                  "speedup_vs_static": static_ms / lat if lat > 0 else None,
                                  "affected_frac": st["affected"] / g.n,
                                  "changed": st["changed"], "passes": st["passes"], "q": q}),
                      file=out, flush=True)
                del h


def temporal_stream(scale: int = 20, edge_factor: int = 16, batches: int = 100, fracs=(1e-5, 1e-4, 1e-3),
                    seed: int = 1, out=sys.stdout):
    """The paper's protocol for temporal graphs (Sec. 5.1.3, 5.1.4) on a
    synthetic stand-in (``inputs.temporal_stream``): the edges of an R-MAT
    graph arrive in a seeded random order, the first 90 % are loaded, then
    `batches` consecutive batches of round(f * |E_T|) updates follow for each
    f in `fracs` (80 % insertions of the next arrivals, 20 % deletions of
    present edges).  Static Leiden on the preloaded graph gives every mode
    the same starting membership; ND, DS and DF then follow the whole stream
    on their own handles.  Per (f, mode): latency p50/p99 (graph update
    excluded), the speedup of p50 over static Leiden on the final graph and
    the final modularity next to static's.  (The DF updates of such a
    stream are compared with the serial oracle from the same membership in
    tests/test_gpu_fullsize.py.)"""
    L = _leiden()
    gT = gen.rmat(scale, edge_factor, seed=seed)
    for f in fracs:
        g0, stream = gen.temporal_stream(gT, f, batches, seed=seed + 17)
        dbs = [L.make_batch(b.del_u, b.del_v, b.ins_u, b.ins_v, b.ins_w) for b in stream]
        h0 = _handle(L, g0)
        C0, _, _ = L.leiden_static(h0)
        C0 = C0.clone()
        del h0
        res = {}
        for mode in MODES:
            h = _handle(L, g0)
            L.leiden_set_state(h, C0)
            lat, q = [], None
            for db in dbs:
                _, q, st, _ = L.leiden_update(h, db, mode)
                lat.append(st["ms_total"] - st["ms_apply"])
            res[mode] = (lat, q)
            if mode == "df":
                off, idx, w = L.leiden_get_graph(h)
            del h
        hs = _handle(L, gen.CSR(g0.n, off.cpu().numpy(), idx.cpu().numpy(), w.cpu().numpy()))
        sms, sq = [], []
        for _ in range(3):
            _, q, st = L.leiden_static(hs)
            sms.append(st["ms_total"])
            sq.append(q)
        del hs
        static_ms = float(np.median(sms[1:]))
        for mode in MODES:
            lat, q = res[mode]
            p50 = float(np.percentile(lat, 50))
            print(json.dumps({"kind": "stream", "frac": f, "mode": mode, "batches": len(dbs),
                              "batch": int(len(stream[0].ins_u) + len(stream[0].del_u)) if stream else 0,
                              "ms_p50": p50, "ms_p99": float(np.percentile(lat, 99)),
                              "ms_mean": float(np.mean(lat)), "static_ms": static_ms,
                              "speedup_vs_static": static_ms / p50 if p50 > 0 else None,
                              "q_final": q, "q_static_final": float(np.mean(sq)),
                              "dq_vs_static": q - float(np.mean(sq))}), file=out, flush=True)


def served(graphs: int = 256, nmin: float = 1e3, nmax: float = 1e7, requests: int = 768, slots: int = 8,
           fleet_max: int = 65536, loads=(0.5, 0.8, 1.0), budget_gb: float = 160.0, seed: int = 1,
           out=sys.stdout):
    """The served batched workload: `graphs` resident dynamic graphs with
    vertex counts log-uniform in [nmin, nmax] (even-indexed R-MAT with edge
    factor 8, odd-indexed planted partitions of 64-vertex blocks with about
    6.3 intra- and 4 inter-block neighbours per vertex; generated on the
    device), and `requests` DF update requests, each on a uniformly chosen
    graph with a batch of log-uniform 1e2..1e6 updates (80 % insertions)
    capped at 0.1 |E| of that graph; a graph's requests apply in order.
    Graphs with at most `fleet_max` vertices are served as jobs of one fleet
    (gathered into shared persistent launches), the others as handles
    (asynchronous mode, working buffers released after every call).

    Forms, each from the same starting memberships (static Leiden):
      * sequential: plain per-graph leiden_update calls, one after another
        on one stream (every graph as a handle);
      * saturation: the server (`slots` workers, memory budget
        `budget_gb`), every request queued at once - its throughput is the
        closed-loop saturation rate mu;
      * poisson: requests arriving as a Poisson process at each offered load
        rho * mu, latency measured from arrival to completion.
    One JSON line per form: updates/s, requests/s, latency p50/p99 and the
    mean final modularity over the graphs."""
    L = _leiden()
    import torch
    rng = np.random.default_rng(seed)
    ns = [int(round(np.exp(rng.uniform(np.log(nmin), np.log(nmax))))) for _ in range(graphs)]
    t = time.time()
    G = []
    for k, n in enumerate(ns):
        if k % 2 == 0:
            scale = max(1, int(np.ceil(np.log2(n))))
            G.append(gen.rmat_device(scale, 8, seed=seed + k, n=n))
        else:
            G.append(gen.planted_device(n, 64, 6.3, 4.0, seed=seed + k))
    torch.cuda.synchronize()
    entries = int(sum(g[2].numel() for g in G))
    owner = rng.integers(0, graphs, requests)
    size = np.exp(rng.uniform(np.log(1e2), np.log(1e6), requests))
    per = {k: [] for k in range(graphs)}
    for r in range(requests):
        k = int(owner[r])
        per[k].append(max(1, int(min(size[r], 0.1 * G[k][2].numel()))))
    streams = {k: gen.batch_stream_device(G[k][0], G[k][1], G[k][2], per[k], len(per[k]), seed=seed + 500 + k)
               for k in range(graphs) if per[k]}
    order, nxt = [], {k: 0 for k in streams}
    for r in range(requests):
        k = int(owner[r])
        order.append((k, streams[k][nxt[k]]))
        nxt[k] += 1
    total = int(sum(int(b[0].numel() + b[2].numel()) for _, b in order))
    small = [k for k in range(graphs) if ns[k] <= fleet_max]
    large = [k for k in range(graphs) if ns[k] > fleet_max]
    slot_of = {k: j for j, k in enumerate(small)}
    print(json.dumps({"kind": "serve_setup", "graphs": graphs, "vertices": int(sum(ns)), "entries": entries,
                      "requests": requests, "updates": total, "fleet_graphs": len(small),
                      "handle_graphs": len(large), "setup_s": round(time.time() - t, 1)}), file=out, flush=True)

    trim = L.leiden_default_params(trim=1)

    def make_fleet():
        fl = L.Fleet([(G[k][1], G[k][2], G[k][3]) for k in small])
        res, _ = fl.run([(j, "static", None) for j in range(len(small))], want_membership=False)
        assert all(r[2] == 0 for r in res)
        return fl

    base = {}
    t = time.time()
    fl0 = make_fleet()
    for j, k in enumerate(small):
        base[k] = fl0.get_state(j)[0].clone()
    fl0.close()
    for k in large:
        h = L.leiden_create(G[k][1], G[k][2], G[k][3], trim)
        base[k] = L.leiden_static(h, want_q=False)[0].clone()
        del h
    torch.cuda.synchronize()
    print(json.dumps({"kind": "serve_static", "seconds": round(time.time() - t, 1)}), file=out, flush=True)

    def handles(keys):
        hs = {}
        for k in keys:
            h = L.leiden_create(G[k][1], G[k][2], G[k][3], trim)
            L.leiden_set_state(h, base[k])
            hs[k] = h
        torch.cuda.synchronize()
        return hs

    def mean_q(hs, fl):
        qs = []
        for k, h in hs.items():
            qs.append(L.leiden_modularity(*L.leiden_get_graph(h), L.leiden_get_state(h)[0]))
        if fl is not None:
            for j, k in enumerate(small):
                qs.append(L.leiden_modularity(*fl.get_graph(j), fl.get_state(j)[0]))
        return float(np.mean(qs))

    def report(form, wall, lats, hs, fl, extra=None):
        rec = {"kind": "serve", "form": form, "wall_s": round(wall, 3), "updates_per_s": total / wall,
               "requests_per_s": requests / wall, "latency_p50_ms": float(np.percentile(lats, 50)),
               "latency_p99_ms": float(np.percentile(lats, 99)), "q_mean": mean_q(hs, fl)}
        if extra:
            rec.update(extra)
        print(json.dumps(rec), file=out, flush=True)
        return rec

    # plain per-graph calls, one after another (latency from time 0, as if all
    # requests were queued at once)
    hs = handles(range(graphs))
    t0 = time.perf_counter()
    lats = []
    for k, b in order:
        L.leiden_update(hs[k], b, "df", want_q=False)
        lats.append((time.perf_counter() - t0) * 1e3)
    wall = time.perf_counter() - t0
    report("sequential", wall, lats, hs, None)
    del hs
    torch.cuda.empty_cache()

    def serve(arrivals):
        hs = handles(large)
        fl = make_fleet()
        sv = L.Server(slots=slots, memory_budget=int(budget_gb * (1 << 30)))
        t0 = time.perf_counter()
        ids = []
        for (k, b), at in zip(order, arrivals):
            now = time.perf_counter() - t0
            if at > now:
                time.sleep(at - now)
            if k in slot_of:
                ids.append(sv.submit_fleet(fl, slot_of[k], b, "df"))
            else:
                ids.append(sv.submit(hs[k], b, "df"))
        lats, svc = [], []
        for rid in ids:
            st, _, _, _, lat, sm = sv.wait(rid)
            assert st == 0, st
            lats.append(lat)
            svc.append(sm)
        wall = time.perf_counter() - t0
        sv.close()
        return hs, fl, wall, lats

    hs, fl, wall, lats = serve([0.0] * requests)
    sat = report("saturation", wall, lats, hs, fl, {"slots": slots, "budget_gb": budget_gb})
    del hs
    fl.close()
    mu = requests / wall
    for rho in loads:
        gaps = rng.exponential(1.0 / (rho * mu), requests)
        arrivals = np.cumsum(gaps) - gaps[0]
        hs, fl, wall, lats = serve(list(arrivals))
        report(f"poisson_{rho:g}", wall, lats, hs, fl, {"offered_requests_per_s": rho * mu})
        del hs
        fl.close()
    return sat


def fleet_vs_calls(graphs: int = 512, nmin: float = 1e3, nmax: float = 3e4, frac_min: float = 1e-3,
                   frac_max: float = 1e-2, rounds: int = 3, seed: int = 1, variant: int | None = None,
                   out=sys.stdout):
    """Many small dynamic graphs with uneven batches, three ways on the same
    GPU from the same starting memberships: plain per-graph leiden_update
    calls one after another (default asynchronous mode), leiden_update_many
    (concurrent streams), and the fused engine (every graph's update in one
    persistent launch per round).  Graphs: n log-uniform in [nmin, nmax],
    even-indexed R-MAT with edge factor 8, odd-indexed planted partitions
    (64-vertex blocks); each round gives every graph a DF batch of
    log-uniform f |E| updates, f in [frac_min, frac_max].  One JSON line per
    form: graph updates per second, edge updates per second, and the mean
    modularity after the last round; the fused engine's result is the serial
    sweep's (the oracle's serial mode)."""
    L = _leiden()
    import torch
    rng = np.random.default_rng(seed)
    gs = []
    for k in range(graphs):
        n = int(round(np.exp(rng.uniform(np.log(nmin), np.log(nmax)))))
        if k % 2 == 0:
            _, off, idx, w = gen.rmat_device(max(1, int(np.ceil(np.log2(n)))), 8, seed=seed + k, n=n)
        else:
            _, off, idx, w = gen.planted_device(n, 64, 6.3, 4.0, seed=seed + k)
        gs.append((off, idx, w))
    streams = []
    for k, (off, idx, w) in enumerate(gs):
        sizes = [max(1, int(round(np.exp(rng.uniform(np.log(frac_min), np.log(frac_max))) * idx.numel() / 2)))
                 for _ in range(rounds)]
        streams.append(gen.batch_stream_device(off.numel() - 1, off, idx, sizes, rounds, seed=seed + 1000 + k))
    updates = sum(int(b[0].numel() + b[2].numel()) for st in streams for b in st)
    entries = sum(int(g[1].numel()) for g in gs)
    print(json.dumps({"kind": "fleet_setup", "graphs": graphs, "entries": int(entries), "rounds": rounds,
                      "updates": updates}), file=out, flush=True)
    fl = L.Fleet(gs)
    if variant is not None:
        fl.set_variant(variant)
    t0 = time.perf_counter()
    res, ms_static = fl.run([(k, "static", None) for k in range(graphs)], want_membership=True)
    wall_static = time.perf_counter() - t0
    base = [r[0].clone() for r in res]
    print(json.dumps({"kind": "fleet_static", "launch_ms": ms_static, "wall_s": wall_static}), file=out, flush=True)

    def q_mean(getter):
        return float(np.mean([L.leiden_modularity(*getter(k)) for k in range(graphs)]))

    # fused: one launch per round
    ms, t0 = [], time.perf_counter()
    for r in range(rounds):
        res, m = fl.run([(k, "df", streams[k][r]) for k in range(graphs)], want_membership=False)
        assert all(x[2] == 0 for x in res)
        ms.append(m)
    wall = time.perf_counter() - t0
    q = q_mean(lambda k: (*fl.get_graph(k), fl.get_state(k)[0]))
    print(json.dumps({"kind": "fleet", "form": "fused", "wall_s": wall, "launch_ms": ms,
                      "graph_updates_per_s": graphs * rounds / wall, "updates_per_s": updates / wall,
                      "q_mean": q}), file=out, flush=True)
    fl.close()

    def handles():
        hs = [L.leiden_create(*g) for g in gs]
        for h, C in zip(hs, base):
            L.leiden_set_state(h, C)
        torch.cuda.synchronize()
        return hs

    hs = handles()
    t0 = time.perf_counter()
    for r in range(rounds):
        for k in range(graphs):
            L.leiden_update(hs[k], streams[k][r], "df", want_q=False)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    q = q_mean(lambda k: (*L.leiden_get_graph(hs[k]), L.leiden_get_state(hs[k])[0]))
    print(json.dumps({"kind": "fleet", "form": "sequential_calls", "wall_s": wall,
                      "graph_updates_per_s": graphs * rounds / wall, "updates_per_s": updates / wall,
                      "q_mean": q}), file=out, flush=True)
    del hs
    hs = handles()
    t0 = time.perf_counter()
    for r in range(rounds):
        res = L.leiden_update_many(hs, [streams[k][r] for k in range(graphs)], ["df"] * graphs, want_q=False,
                                   max_parallel=16)
        assert all(x[3] == 0 for x in res)
    wall = time.perf_counter() - t0
    q = q_mean(lambda k: (*L.leiden_get_graph(hs[k]), L.leiden_get_state(hs[k])[0]))
    print(json.dumps({"kind": "fleet", "form": "update_many", "wall_s": wall,
                      "graph_updates_per_s": graphs * rounds / wall, "updates_per_s": updates / wall,
                      "q_mean": q}), file=out, flush=True)


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
    t.add_argument("--fracs", type=float, nargs="+", default=[1e-5, 1e-4, 1e-3])
    v = sub.add_parser("serve")
    v.add_argument("--graphs", type=int, default=256)
    v.add_argument("--nmax", type=float, default=1e7)
    v.add_argument("--requests", type=int, default=768)
    v.add_argument("--slots", type=int, default=8)
    v.add_argument("--fleet-max", type=int, default=65536)
    v.add_argument("--budget-gb", type=float, default=160.0)
    f = sub.add_parser("fleet")
    f.add_argument("--graphs", type=int, default=512)
    f.add_argument("--nmax", type=float, default=3e4)
    f.add_argument("--rounds", type=int, default=3)
    f.add_argument("--variant", type=int, default=None)
    a = ap.parse_args(argv)
    t0 = time.time()
    if a.cmd == "sweep":
        batch_sweep(a.scale, a.edge_factor, tuple(a.fracs), a.reps)
    elif a.cmd == "stream":
        temporal_stream(a.scale, a.edge_factor, a.batches, tuple(a.fracs))
    elif a.cmd == "fleet":
        fleet_vs_calls(a.graphs, 1e3, a.nmax, rounds=a.rounds, variant=a.variant)
    else:
        served(a.graphs, 1e3, a.nmax, a.requests, a.slots, a.fleet_max, budget_gb=a.budget_gb)
    print(json.dumps({"kind": "done", "seconds": round(time.time() - t0, 1)}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
