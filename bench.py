#!/usr/bin/env python3
"""Dynamic Frontier Leiden update benchmark on one MI355X.

Workload (synthetic, seeded): RMAT scale 22, edge factor 16 with
(a, b, c) = (0.57, 0.19, 0.19), symmetrised, self-loops and repeated edges
removed, vertex ids randomly permuted, unit float32 weights (4,194,304
vertices, ~128.3M directed CSR entries).  Static Leiden runs once; then a
stream of batches, each of round(f * |E|) undirected updates (80% insertions
of uniformly random non-edges, 20% deletions of uniformly chosen existing
edges; Sec. 5.1.4), is applied with the Dynamic Frontier front-end
(Sec. 4.5, Alg. "dynamicFrontier").  The batches of the whole run are drawn
up front (disjoint, so they apply one after another) and copied to HBM before
any timing.

One step = one leiden_update(mode=DF) call through the C ABI: batch
validation and graph update, DF marking, changedCommunities, updateWeights,
the pass loop (local-moving, refinement, aggregation), final relabel, and the
modularity of the result (Eq. 1).  `value` is |E^t| / (wall time per step)
over the timed steps; latencies p50/p99 come from HIP events inside the
library and exclude the graph update, which the paper does not time
(Sec. 5.1.4).  Static Leiden on the same graph is timed for the comparison.
Modularity: the mean over the last five updates against the mean of
--static-reps static runs on the final graph (both are asynchronous heuristics
whose results vary from run to run by about 1e-3).

roofline: the timed kernel (leiden_params.profile) with the largest share of
the timed steps; achieved = algorithmic bytes / event-timed duration.
Algorithmic bytes per unit: hub gather 12 B per scanned entry (id, weight,
community of the neighbour); aggregation merge 12 B per entry plus 12 B per
member vertex (community-CSR entry and its community); modularity scan 12 B
per entry plus 4 B per vertex; graph-update merge 16 B per entry (read and
write of id + weight) plus 16 B per vertex (old and new offsets); asynchronous
local-moving sweep 12 B per scanned edge (id, weight, community of the
neighbour) plus 34 B per evaluated vertex (list entry, two offsets, range and
processed flags, community, K); Sigma reads and neighbour marks are not
counted (a lower bound).

cpu_baseline: the serial C oracle (test infrastructure) on the same graph and
first batch: its own static run (untimed preparation), then one DF update,
timed; edges/s = |E^t| / that time; one host thread.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

METRIC = "DF-Leiden update latency & edges/s vs static Leiden at ΔQ≤1e-3; p50/p99"
HBM_PEAK_GBS = 8000.0
BYTES_PER_UNIT = {  # (per entry, per vertex)
    "hub_gather": (12.0, 0.0),
    "agg_merge": (12.0, 12.0),
    "mod_scan": (12.0, 4.0),
    "batch_merge": (16.0, 16.0),
    "move_sweep": (12.0, 34.0),
}
PROF_KERNEL_NAMES = {  # symbol of each timed kernel, as rocprofv3 lists it
    "hub_gather": "lk::k_hub_gather(lk::MoveArgs)",
    "agg_merge": "lk::k_agg_items(lk::AggArgs, long)",
    "mod_scan": "lk::k_mod_edges",
    "batch_merge": "lk::k_batch_apply_old(lk::BatchArgs)",
    "move_sweep": "lk::k_move_async",  # both launch shapes, <4, 512> and <2, 2048>
}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def pct(xs, q):
    return float(np.percentile(np.asarray(xs, dtype=np.float64), q)) if len(xs) else None


def ratio(a, b):
    return round(a / b, 4) if b else None


def measured_traffic(kernel: str):
    """Bytes per launch of `kernel` from the committed counter runs
    (profiles/traffic.json: FETCH_SIZE and WRITE_SIZE scaled by a 1 GiB copy),
    or None when there is none for the kernels as they are now (the entry
    records a hash of the kernel sources it was measured on)."""
    import glob
    import hashlib
    path = os.path.join(HERE, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    entry = json.load(open(path)).get(kernel)
    if not entry:
        return None
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(HERE, "paper_2405_11658_amd", "csrc", "*"))):
        with open(p, "rb") as f:
            h.update(f.read())
    return entry["bytes_per_launch"] if entry.get("source_sha256") == h.hexdigest() else None


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--scale", type=int, default=22)
    ap.add_argument("--edge-factor", type=int, default=16)
    ap.add_argument("--frac", type=float, default=1e-4, help="batch size as a fraction of |E|")
    ap.add_argument("--mode", default="df", choices=["df", "ds", "nd"])
    ap.add_argument("--static-reps", type=int, default=3)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="end with a 1 GiB device-to-device copy (reference for counter runs)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only (asked for --gpus {args.gpus}); the library has no "
              "multi-GPU path", file=sys.stderr)
        return 2
    if args.steps < 1 or args.warmup < 0:
        print("bench.py: --steps must be >= 1 and --warmup >= 0", file=sys.stderr)
        return 2

    import torch
    from paper_2405_11658_amd import inputs as gen
    from paper_2405_11658_amd import leiden as L

    if not torch.cuda.is_available():
        raise SystemExit("bench.py: no HIP device visible")
    torch.cuda.set_device(0)
    L.load()

    t = time.time()
    g = gen.rmat(args.scale, args.edge_factor, seed=args.seed)
    log(f"graph: RMAT scale {args.scale} ef {args.edge_factor}: n={g.n} entries={g.nnz} ({time.time() - t:.1f}s)")
    B = gen.batch_count(g.nnz, args.frac)
    nb = args.warmup + args.steps
    t = time.time()
    batches_h = gen.batch_stream(g, B, nb, seed=args.seed + 1000)
    log(f"batches: {nb} x {B} updates ({time.time() - t:.1f}s)")

    h = L.leiden_create(g.off, g.idx, g.w, L.leiden_default_params())
    batches = [L.make_batch(b.del_u, b.del_v, b.ins_u, b.ins_v, b.ins_w) for b in batches_h]
    torch.cuda.synchronize()

    # static Leiden on the initial graph (the first run also warms up)
    static_ms = []
    q_static0 = None
    for r in range(max(1, args.static_reps)):
        _, q_static0, st = L.leiden_static(h)
        static_ms.append(st["ms_total"])
        log(f"static #{r}: {st['ms_total']:.2f} ms Q={q_static0:.6f} passes={st['passes']}")
    static_ms_timed = static_ms[1:] if len(static_ms) > 1 else static_ms

    q_first = None
    for k in range(args.warmup):
        _, q, st, _ = L.leiden_update(h, batches[k], args.mode)
        if k == 0:
            q_first = q
        log(f"warmup {k}: {st['ms_total']:.2f} ms Q={q:.6f}")

    L.leiden_set_params(h, L.leiden_default_params(profile=1))
    lat, lat_all, ents, qs = [], [], [], []
    prof = {name: {"launches": 0, "ms": 0.0, "entries": 0, "vertices": 0} for name in L.PROF_KERNELS}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        _, q, st, _ = L.leiden_update(h, batches[args.warmup + k], args.mode)
        lat.append(st["ms_total"] - st["ms_apply"])
        lat_all.append(st["ms_total"])
        qs.append(q)
        for name, v in st["prof"].items():
            for key in v:
                prof[name][key] += v[key]
        ents.append(st["level_entries"][0] if st["passes"] else 0)
        log(f"step {k}: {st['ms_total']:.2f} ms (apply {st['ms_apply']:.2f}) Q={q:.6f} "
            f"affected={st['affected']} passes={st['passes']}")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    L.leiden_set_params(h, L.leiden_default_params())
    if q_first is None:
        q_first = qs[0]

    ms_per_step = wall * 1e3 / args.steps
    entries = float(np.mean(ents))
    value = entries / (ms_per_step / 1e3)

    # static Leiden on the final graph: modularity reference for the updates.
    # Both sides are asynchronous heuristics whose modularity varies from run
    # to run by about 1e-3, so the comparison is of means: the last five
    # updates against several static runs on the final graph.
    q_static_final = []
    for r in range(max(1, args.static_reps)):
        _, q, st = L.leiden_static(h)
        q_static_final.append(q)
        log(f"static on final graph #{r}: {st['ms_total']:.2f} ms Q={q:.6f}")
    q_upd_tail = float(np.mean(qs[-5:]))
    q_stat_mean = float(np.mean(q_static_final))

    # roofline of the timed kernel with the largest total time
    dom = max(prof, key=lambda k: prof[k]["ms"])
    pd = prof[dom]
    roofline = None
    if pd["launches"] > 0 and pd["ms"] > 0:
        be, bv = BYTES_PER_UNIT[dom]
        bytes_per_launch = (be * pd["entries"] + bv * pd["vertices"]) / pd["launches"]
        avg_ms = pd["ms"] / pd["launches"]
        achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
        roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(PROF_KERNEL_NAMES[dom]),
                    "kernel": PROF_KERNEL_NAMES[dom], "avg_launch_us": round(avg_ms * 1e3, 2),
                    "launches_per_step": pd["launches"] / args.steps,
                    "algorithmic_bytes_per_launch": round(bytes_per_launch),
                    "share_of_step": round(pd["ms"] / args.steps / ms_per_step, 4)}

    cpu = None
    q_oracle_first = None
    if not args.no_cpu_baseline:
        import oracle
        oracle.build()
        og = oracle.as_graph(g.n, g.off, g.idx, g.w)
        t = time.perf_counter()
        ost, _ = oracle.static(og, oracle.make_params())
        t_static = time.perf_counter() - t
        log(f"oracle static: {t_static:.1f}s")
        b = batches_h[0]
        t = time.perf_counter()
        ost2, _, _, _ = oracle.update(ost, oracle.Batch(b.del_u, b.del_v, b.ins_u, b.ins_v, b.ins_w),
                                      args.mode, oracle.make_params())
        t_upd = time.perf_counter() - t
        q_oracle_first = oracle.modularity(ost2.g, ost2.C)
        log(f"oracle {args.mode} update: {t_upd:.2f}s Q={q_oracle_first:.6f}")
        cpu = {"value": ratio(ost2.g.nnz, t_upd), "unit": "edges/s", "cores": 1, "kind": "oracle",
               "sample": (f"one {args.mode.upper()} update (batch 0, {B} updates) of the serial oracle on "
                          f"the same graph after its own static run ({t_static:.1f}s, untimed); "
                          f"update {t_upd:.2f}s; host CPU {cpu_model()}, os.cpu_count()={os.cpu_count()}")}

    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("1 GiB calibration copy done")

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"rmat{args.scale}_ef{args.edge_factor}_{args.mode}_f{args.frac:g}",
                   "n": g.n, "entries": int(g.nnz), "batch_updates": B, "mode": args.mode,
                   "hub_slices": 64},
        "latency_ms": {"p50": round(pct(lat, 50), 3), "p99": round(pct(lat, 99), 3),
                       "mean": round(float(np.mean(lat)), 3)},
        "latency_with_graph_update_ms": {"p50": round(pct(lat_all, 50), 3), "p99": round(pct(lat_all, 99), 3)},
        "updates_per_s": ratio(B * 1e3, pct(lat, 50)),
        "static_ms": {"p50": round(pct(static_ms_timed, 50), 3), "reps": len(static_ms_timed)},
        "speedup_vs_static": ratio(pct(static_ms_timed, 50), pct(lat, 50)),
        "modularity": {"update_last": qs[-1], "update_last5_mean": q_upd_tail,
                       "static_final_graph": q_static_final, "static_final_mean": q_stat_mean,
                       "dq_update_vs_static": q_upd_tail - q_stat_mean,
                       "update_first": q_first, "oracle_update_first": q_oracle_first,
                       "dq_vs_oracle": (q_first - q_oracle_first) if q_oracle_first is not None else None,
                       "static_initial": q_static0},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
