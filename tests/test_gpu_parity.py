"""GPU parity: the HIP library (through the C ABI) against the CPU oracle.

Bars (integer edge weights, so every FP64 sum is exact and order-free):
  * modularity: relative difference <= 1e-9;
  * aggregation for a given membership: identical super-vertex matrix;
  * batch apply: identical CSR; marking (DF/DS/ND) and changed flags: identical;
  * synchronous mode: identical membership and identical per-pass statistics;
  * default (atomic-sum) mode: modularity within 1e-3 of the oracle's serial
    asynchronous run, and the Leiden invariants.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2405_11658_amd import inputs as gen
from paper_2405_11658_amd import leiden as L

from .gpu_common import canon_rows, dev_batch, ob, og, say, sync_params, to_np
from .helpers import communities_connected, same_partition

pytestmark = pytest.mark.gpu


def _graphs_small():
    return [
        ("clique_ring_4x5", gen.clique_ring(4, 5)),
        ("gnp60_int", gen.gnp(60, 0.12, seed=5, weights="int")),
        ("planted1024", gen.planted_partition(1024, 16, 0.15, 0.004, seed=7)),
    ]


@pytest.mark.parametrize("name,g", _graphs_small() + [("C1_planted4096", gen.planted_partition(4096, 64, 0.1, 0.001, seed=1))])
def test_modularity_parity(name, g):
    rng = np.random.default_rng(0)
    for k in (1, 7, g.n // 3 + 1, g.n):
        C = rng.integers(0, k, g.n).astype(np.int32)
        say("modularity", name, "k", k)
        q = L.leiden_modularity(g.off, g.idx, g.w, C)
        qo = oracle.modularity(og(g), C)
        assert abs(q - qo) <= 1e-9 * max(1.0, abs(qo)), (q, qo)


def test_modularity_edge_cases():
    say("modularity edge cases")
    g = gen.from_edges(5, [], [])
    assert L.leiden_modularity(g.off, g.idx, g.w, np.arange(5)) == 0.0
    with pytest.raises(L.LeidenError):
        L.leiden_modularity(g.off, g.idx, g.w, np.full(5, 7))


@pytest.mark.parametrize("name,g", _graphs_small() + [("rmat12", gen.rmat(12, 8, seed=3))])
def test_aggregate_parity(name, g):
    rng = np.random.default_rng(1)
    for k in (1, 5, max(2, g.n // 10), g.n):
        C = rng.integers(0, k, g.n).astype(np.int32)
        _, C = np.unique(C, return_inverse=True)
        C = C.astype(np.int32)
        ncomm = int(C.max()) + 1
        say("aggregate", name, "ncomm", ncomm)
        off, idx, w = L.leiden_aggregate(g.off, g.idx, g.w, C, ncomm)
        ref = oracle.aggregate(og(g), C, ncomm)
        assert canon_rows(to_np(off), to_np(idx), to_np(w)) == canon_rows(ref.off, ref.idx, ref.w)


def test_aggregate_parity_long_rows():
    """Memberships whose communities own thousands of entries each (rows that
    span several 4096-entry tiles of the segmented sort, runs of one neighbour
    community that cross tile boundaries) mixed with small ones, on an RMAT
    graph with hubs."""
    g = gen.rmat(16, 16, seed=5)
    rng = np.random.default_rng(2)
    deg = np.diff(g.off)
    for k in (2, 64, 700):
        C = rng.integers(0, k, g.n).astype(np.int32)
        # the hubs and a block of vertices get communities of their own
        C[np.argsort(deg)[-50:]] = np.arange(k, k + 50, dtype=np.int32)
        C[: g.n // 8] = rng.integers(k + 50, k + 50 + g.n // 16, g.n // 8)
        _, C = np.unique(C, return_inverse=True)
        C = C.astype(np.int32)
        ncomm = int(C.max()) + 1
        say("aggregate long rows rmat16 ncomm", ncomm)
        off, idx, w = L.leiden_aggregate(g.off, g.idx, g.w, C, ncomm)
        ref = oracle.aggregate(og(g), C, ncomm)
        assert np.array_equal(to_np(off), ref.off)
        assert canon_rows(to_np(off), to_np(idx), to_np(w)) == canon_rows(ref.off, ref.idx, ref.w)


def _static_pair(g, params_gpu, params_or):
    h = L.leiden_create(g.off, g.idx, g.w, params_gpu)
    C, q, st = L.leiden_static(h)
    ost, ostats = oracle.static(og(g), params_or)
    return h, to_np(C), q, st, ost, ostats


STAT_KEYS = ("passes", "move_iters", "refine_rounds", "level_vertices", "level_entries", "communities",
             "refined_vertices", "affected", "changed", "moves_pass0")


@pytest.mark.parametrize("name,g", _graphs_small() + [
    ("C1_planted4096", gen.planted_partition(4096, 64, 0.1, 0.001, seed=1)),
    ("rmat14_ef8", gen.rmat(14, 8, seed=2)),
    ("grid64", gen.grid2d(64, 0.05, 0.02, seed=1)),
])
def test_static_sync_bit_exact(name, g):
    say("static sync", name, "n", g.n, "nnz", g.nnz)
    h, C, q, st, ost, ostats = _static_pair(g, sync_params(), oracle.make_params(sync=True))
    assert np.array_equal(C, ost.C), name
    for k in STAT_KEYS:
        assert st[k] == ostats[k], (k, st[k], ostats[k])
    qo = oracle.modularity(og(g), ost.C)
    assert abs(q - qo) <= 1e-9 * max(1.0, abs(qo))
    Cs, K, S, m2 = L.leiden_get_state(h)
    assert np.array_equal(to_np(K), ost.K) and np.array_equal(to_np(S), ost.Sig) and m2 == ost.M2


def test_static_hub_bucket_sync_bit_exact():
    g = gen.rmat(16, 16, seed=4)
    deg = np.diff(g.off)
    say("static sync rmat16 maxdeg", int(deg.max()))
    assert deg.max() > 2048  # exercises the global-table bucket
    h, C, q, st, ost, ostats = _static_pair(g, sync_params(), oracle.make_params(sync=True))
    assert np.array_equal(C, ost.C)
    for k in STAT_KEYS:
        assert st[k] == ostats[k], (k, st[k], ostats[k])


@pytest.mark.parametrize("mode", ["nd", "ds", "df"])
@pytest.mark.parametrize("name,g,frac", [
    ("C1_planted4096", gen.planted_partition(4096, 64, 0.1, 0.001, seed=1), 1e-3),
    ("planted1024_big_batch", gen.planted_partition(1024, 16, 0.15, 0.004, seed=7), 2e-2),
    ("rmat13", gen.rmat(13, 8, seed=6), 1e-3),
])
def test_update_sync_bit_exact(mode, name, g, frac):
    h = L.leiden_create(g.off, g.idx, g.w, sync_params())
    L.leiden_static(h)
    state, _ = oracle.static(og(g), oracle.make_params(sync=True))
    C0 = to_np(L.leiden_get_state(h)[0])
    assert np.array_equal(C0, state.C)
    for seed in range(3):
        b = gen.random_batch(gen.CSR(state.g.n, state.g.off, state.g.idx, state.g.w),
                             gen.batch_count(state.g.nnz, frac), seed=seed)
        say("update sync", name, mode, "seed", seed, "batch", b.size)
        C, q, st, tr = L.leiden_update(h, dev_batch(b), mode, trace=True)
        gt, dw = oracle.apply_batch(state.g, ob(b))
        off, idx, w = L.leiden_get_graph(h)
        assert np.array_equal(to_np(off), gt.off) and np.array_equal(to_np(idx), gt.idx)
        assert np.array_equal(to_np(w), gt.w)
        dV, rng, dC = oracle.mark(mode, gt, ob(b), state.C, state.K, state.Sig, state.M2)
        assert np.array_equal(to_np(tr["affected"]), dV)
        assert np.array_equal(to_np(tr["in_range"]), rng)
        assert np.array_equal(to_np(tr["changed"]), dC)
        new, dV2, dC2, ostats = oracle.update(state, ob(b), mode, oracle.make_params(sync=True))
        assert np.array_equal(to_np(C), new.C), (name, mode, seed)
        for k in STAT_KEYS:
            assert st[k] == ostats[k], (k, st[k], ostats[k])
        Cs, K, S, m2 = L.leiden_get_state(h)
        assert np.array_equal(to_np(K), new.K) and np.array_equal(to_np(S), new.Sig) and m2 == new.M2
        state = new


def test_update_from_installed_state():
    """set_state installs the oracle's asynchronous membership; one DF update
    from identical state must then match the oracle's synchronous update."""
    g = gen.planted_partition(2048, 32, 0.12, 0.002, seed=9)
    state, _ = oracle.static(og(g), oracle.make_params(sync=False))
    h = L.leiden_create(g.off, g.idx, g.w, sync_params())
    L.leiden_set_state(h, state.C)
    Cs, K, S, m2 = L.leiden_get_state(h)
    assert np.array_equal(to_np(K), state.K) and np.array_equal(to_np(S), state.Sig) and m2 == state.M2
    b = gen.random_batch(g, 20, seed=3)
    say("update from installed state")
    C, q, st, _ = L.leiden_update(h, dev_batch(b), "df")
    new, _, _, _ = oracle.update(state, ob(b), "df", oracle.make_params(sync=True))
    assert np.array_equal(to_np(C), new.C)


def test_default_mode_quality_vs_oracle_async():
    """Default mode against the oracle's serial asynchronous run (the paper's
    order) on id-permuted planted-partition graphs (no id locality to favour
    either order): static runs, and DF updates started from the same installed
    state on both sides.  The mean gap Q_gpu - Q_oracle of the six DF
    updates (same membership on both sides) must lie within 1e-3 either way.
    Static runs start from singletons, so the two orders differ from the
    start: relabelling the vertices alone moves the oracle's result by about
    2.5e-3 on these graphs, and single GPU runs of one graph spread by timing
    (12 runs per seed: standard deviation about 1.5e-3, lowest -6.5e-3).  So
    the static gate is on the mean of five runs per seed (fifteen runs;
    measured means of nine runs -1.6e-3 to -2.3e-3; standard error of fifteen
    about 4e-4): at least -3e-3.  Every community connected."""
    gaps, sgaps = [], []
    for seed in (1, 2, 3):
        g = gen.planted_partition(4096, 64, 0.1, 0.001, seed=seed, permute=True)
        ost, _ = oracle.static(og(g))
        qo = oracle.modularity(og(g), ost.C)
        for r in range(5):
            h = L.leiden_create(g.off, g.idx, g.w)
            say("default mode static, planted 4096 permuted, seed", seed, "run", r)
            C, q, st = L.leiden_static(h)
            sgaps.append(q - qo)
            assert communities_connected(og(g), to_np(C))
        state = ost
        for k in range(2):
            L.leiden_set_state(h, state.C)
            b = gen.random_batch(gen.CSR(state.g.n, state.g.off, state.g.idx, state.g.w),
                                 gen.batch_count(state.g.nnz, 1e-3), seed=10 + k)
            say("default mode df, seed", seed, "batch", k)
            C, q, st, _ = L.leiden_update(h, dev_batch(b), "df")
            state, _, _, _ = oracle.update(state, ob(b), "df")
            qo = oracle.modularity(state.g, state.C)
            gaps.append(q - qo)
            assert communities_connected(state.g, to_np(C))
    gaps, sgaps = np.array(gaps), np.array(sgaps)
    say("static Q_gpu - Q_oracle:", np.round(sgaps, 5).tolist(), "DF (same state):", np.round(gaps, 5).tolist(),
        "mean", round(float(gaps.mean()), 5))
    assert abs(gaps.mean()) <= 1e-3, gaps
    assert sgaps.mean() >= -3e-3, sgaps


def test_empty_batch_and_errors():
    g = gen.clique_ring(4, 5)
    h = L.leiden_create(g.off, g.idx, g.w, sync_params())
    e = np.array([], np.int32)
    say("update before static")
    with pytest.raises(L.LeidenError) as ex:
        L.leiden_update(h, L.make_batch(e, e, e, e, np.array([], np.float32)), "df")
    assert ex.value.status == L.ESTATE
    C0, _, _ = L.leiden_static(h)
    say("empty batch df")
    C, q, st, tr = L.leiden_update(h, L.make_batch(e, e, e, e, np.array([], np.float32)), "df", trace=True)
    assert st["affected"] == 0 and int(tr["changed"].sum()) == 0
    assert same_partition(to_np(C), np.repeat(np.arange(4), 5))
    off0, idx0, w0 = [to_np(t) for t in L.leiden_get_graph(h)]
    bad = [
        ([0], [7], [], [], []),              # deleting 0-7, which is not an edge
        ([], [], [0], [1], [1.0]),           # inserting an existing edge
        ([], [], [3], [3], [1.0]),           # self-loop
        ([], [], [0], [20], [1.0]),          # id out of range
        ([], [], [0], [7], [0.0]),           # non-positive weight
        ([], [], [0, 7], [7, 0], [1.0, 1.0]),  # repeated edge
    ]
    for k, (du, dv, iu, iv, iw) in enumerate(bad):
        say("invalid batch", k)
        with pytest.raises(L.LeidenError) as ex:
            L.leiden_update(h, L.make_batch(np.array(du, np.int32), np.array(dv, np.int32),
                                            np.array(iu, np.int32), np.array(iv, np.int32),
                                            np.array(iw, np.float32)), "df")
        assert ex.value.status == L.EINVAL
        off, idx, w = [to_np(t) for t in L.leiden_get_graph(h)]
        assert np.array_equal(off, off0) and np.array_equal(idx, idx0) and np.array_equal(w, w0)


def test_empty_and_edgeless_graphs():
    for n in (0, 1, 7):
        g = gen.from_edges(n, [], [])
        say("edgeless graph", n)
        h = L.leiden_create(g.off, g.idx, g.w)
        C, q, st = L.leiden_static(h)
        assert list(to_np(C)) == list(range(n)) and q == 0.0


def test_create_rejects_bad_graphs():
    say("create rejects")
    with pytest.raises(L.LeidenError):
        L.leiden_create(np.array([0, 2, 2]), np.array([1, 1], np.int32), np.array([1, 1], np.float32))
    with pytest.raises(L.LeidenError):
        L.leiden_create(np.array([0, 1, 2]), np.array([1, 0], np.int32), np.array([1, -1], np.float32))
    # unsorted rows are accepted and sorted by the library
    g = gen.gnp(30, 0.2, seed=1, weights="int")
    perm_idx = g.idx.copy()
    perm_w = g.w.copy()
    for r in range(g.n):
        a, b = g.off[r], g.off[r + 1]
        p = np.random.default_rng(r).permutation(b - a)
        perm_idx[a:b] = g.idx[a:b][p]
        perm_w[a:b] = g.w[a:b][p]
    h = L.leiden_create(g.off, perm_idx, perm_w)
    off, idx, w = [to_np(t) for t in L.leiden_get_graph(h)]
    assert np.array_equal(idx, g.idx) and np.array_equal(w, g.w)


@pytest.mark.parametrize("variant", [1, 2])
@pytest.mark.parametrize("name,g", [
    ("C1_planted4096", gen.planted_partition(4096, 64, 0.1, 0.001, seed=1)),
    ("rmat13", gen.rmat(13, 8, seed=6)),
])
def test_refine_variants_sync_bit_exact(variant, name, g):
    """Full Refine (Sec. 4.2) and no continued passes (Sec. 4.1): static and
    one DF update, identical to the oracle in synchronous mode."""
    h = L.leiden_create(g.off, g.idx, g.w, sync_params(refine_variant=variant))
    prm = oracle.make_params(sync=True, refine_variant=variant)
    say("refine variant", variant, name)
    C, q, st = L.leiden_static(h)
    state, ostats = oracle.static(og(g), prm)
    assert np.array_equal(to_np(C), state.C)
    for k in STAT_KEYS:
        assert st[k] == ostats[k], (k, st[k], ostats[k])
    b = gen.random_batch(g, gen.batch_count(g.nnz, 1e-3), seed=11)
    C, q, st, _ = L.leiden_update(h, dev_batch(b), "df")
    new, _, _, ostats = oracle.update(state, ob(b), "df", prm)
    assert np.array_equal(to_np(C), new.C)
    for k in STAT_KEYS:
        assert st[k] == ostats[k], (k, st[k], ostats[k])
    qo = oracle.modularity(new.g, new.C)
    assert abs(q - qo) <= 1e-9 * max(1.0, abs(qo))


def test_update_many_matches_single_updates():
    """Batched updates of several graphs equal the same updates run one at a
    time (synchronous mode: identical memberships); a malformed batch fails
    alone."""
    graphs = [gen.planted_partition(4096, 64, 0.1, 0.001, seed=1), gen.rmat(13, 8, seed=6),
              gen.grid2d(64, 0.05, 0.02, seed=1), gen.planted_partition(1024, 16, 0.15, 0.004, seed=7)]
    many, single, batches = [], [], []
    for k, g in enumerate(graphs):
        a = L.leiden_create(g.off, g.idx, g.w, sync_params())
        b = L.leiden_create(g.off, g.idx, g.w, sync_params())
        L.leiden_static(a)
        L.leiden_static(b)
        many.append(a)
        single.append(b)
        batches.append(gen.random_batch(g, gen.batch_count(g.nnz, 1e-3), seed=20 + k))
    bad = gen.UBatch(np.array([0], np.int32), np.array([0], np.int32), np.zeros(0, np.int32),
                     np.zeros(0, np.int32), np.zeros(0, np.float32))  # self-loop deletion: invalid
    say("update_many over", len(graphs), "graphs + 1 invalid")
    g5 = gen.clique_ring(4, 5)
    h5 = L.leiden_create(g5.off, g5.idx, g5.w, sync_params())
    L.leiden_static(h5)
    res = L.leiden_update_many(many + [h5], [dev_batch(b) for b in batches] + [dev_batch(bad)],
                               ["df", "ds", "nd", "df", "df"], max_parallel=3)
    assert res[-1][3] == L.EINVAL
    for k, (h, b) in enumerate(zip(single, batches)):
        C, q, st, _ = L.leiden_update(h, dev_batch(b), ["df", "ds", "nd", "df"][k])
        Cm, qm, stm, status = res[k]
        assert status == L.OK
        assert np.array_equal(to_np(Cm), to_np(C)), k
        assert abs(qm - q) <= 1e-12 * abs(q)  # modularity sums with atomics: last bits vary
