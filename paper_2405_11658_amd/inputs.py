"""Seeded synthetic inputs: graphs and batch updates.

This module holds input construction only (no step of the community-detection
method).  Both the GPU path's tests/benchmark and the CPU oracle's tests draw
their inputs from here, so the two sides always see identical data.

Workload shapes follow the paper's evaluation (Sec. 5.1.3 and 5.1.4): undirected
graphs stored with both directions, unit weights, batches of 80% insertions of
uniformly random vertex pairs and 20% deletions of uniformly chosen existing
edges, no new vertices, batch size a fraction of |E|.  The paper's SuiteSparse
and SNAP graphs are not available; planted-partition, R-MAT and 2D-grid graphs
stand in for them.

All randomness comes from ``numpy.random.Generator(PCG64(seed))``.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class CSR:
    n: int
    off: np.ndarray   # int64 [n+1]
    idx: np.ndarray   # int32 [nnz]
    w: np.ndarray     # float32 [nnz]

    @property
    def nnz(self) -> int:
        return int(self.off[-1])


@dataclass
class UBatch:
    """Undirected batch update, each edge listed once."""
    del_u: np.ndarray
    del_v: np.ndarray
    ins_u: np.ndarray
    ins_v: np.ndarray
    ins_w: np.ndarray

    @property
    def size(self) -> int:
        return len(self.del_u) + len(self.ins_u)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def from_edges(n: int, u, v, w=None, keep_self_loops: bool = False) -> CSR:
    """Undirected CSR from an edge list: both directions stored, duplicates merged
    (first weight kept), rows sorted by neighbour id.  A self-loop is stored once."""
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    if w is None:
        w = np.ones(len(u), np.float32)
    w = np.asarray(w, dtype=np.float32)
    if not keep_self_loops:
        m = u != v
        u, v, w = u[m], v[m], w[m]
    loops = u == v
    # canonical undirected key so both orientations share one weight
    a = np.minimum(u, v)
    b = np.maximum(u, v)
    key = a * n + b
    key, first = np.unique(key, return_index=True)
    w = w[first]
    a = key // n
    b = key % n
    loops = a == b
    src = np.concatenate([a, b[~loops]])
    dst = np.concatenate([b, a[~loops]])
    ww = np.concatenate([w, w[~loops]])
    order = np.lexsort((dst, src))
    src, dst, ww = src[order], dst[order], ww[order]
    off = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(src, minlength=n), out=off[1:])
    return CSR(n, off, dst.astype(np.int32), ww.astype(np.float32))


def _csr_from_sorted_unique_keys(n: int, key: np.ndarray) -> CSR:
    src = key // n
    dst = (key % n).astype(np.int32)
    off = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(src, minlength=n), out=off[1:])
    return CSR(n, off, dst, np.ones(len(dst), np.float32))


def _symmetric_csr(n: int, u: np.ndarray, v: np.ndarray) -> CSR:
    """Unit-weight undirected CSR, self-loops and duplicates removed."""
    u = np.asarray(u, np.int64)
    v = np.asarray(v, np.int64)
    m = u != v
    u, v = u[m], v[m]
    key = np.concatenate([u * n + v, v * n + u])
    del u, v
    key = np.unique(key)
    return _csr_from_sorted_unique_keys(n, key)


def planted_partition(n: int = 4096, blocks: int = 64, p_in: float = 0.1, p_out: float = 0.001,
                      seed: int = 1, permute: bool = False) -> CSR:
    """Planted-partition graph: `blocks` contiguous equal blocks; each vertex pair
    is an edge independently with p_in inside a block, p_out across blocks.
    With ``permute`` the vertex ids are relabelled by a seeded permutation (so
    blocks are not contiguous id ranges)."""
    if permute:
        g = planted_partition(n, blocks, p_in, p_out, seed, permute=False)
        perm = _rng(seed + 7919).permutation(n)
        src = np.repeat(np.arange(n), np.diff(g.off))
        return _symmetric_csr(n, perm[src], perm[g.idx])
    rng = _rng(seed)
    bs = n // blocks
    block = np.minimum(np.arange(n) // max(bs, 1), blocks - 1)
    if n <= 20000:
        iu, ju = np.triu_indices(n, k=1)
        same = block[iu] == block[ju]
        p = np.where(same, p_in, p_out)
        keep = rng.random(len(iu)) < p
        return _symmetric_csr(n, iu[keep], ju[keep])
    # large n: per-class edge counts ~ Binomial, then uniform distinct pairs
    us, vs = [], []
    sizes = np.bincount(block, minlength=blocks).astype(np.int64)
    starts = np.concatenate([[0], np.cumsum(sizes)[:-1]])
    n_in_pairs = sizes * (sizes - 1) // 2
    cnt_in = rng.binomial(n_in_pairs, p_in)
    for bidx in range(blocks):
        k = int(cnt_in[bidx])
        if k == 0:
            continue
        s, z = int(starts[bidx]), int(sizes[bidx])
        got = np.empty(0, np.int64)
        while len(got) < k:
            a = rng.integers(0, z, 2 * (k - len(got)) + 16)
            b = rng.integers(0, z, len(a))
            ok = a < b
            got = np.unique(np.concatenate([got, a[ok] * z + b[ok]]))
        got = rng.permutation(got)[:k]
        us.append(s + got // z)
        vs.append(s + got % z)
    total_pairs = n * (n - 1) // 2
    out_pairs = total_pairs - int(n_in_pairs.sum())
    k = int(rng.binomial(out_pairs, p_out))
    got = np.empty(0, np.int64)
    while len(got) < k:
        a = rng.integers(0, n, 2 * (k - len(got)) + 16)
        b = rng.integers(0, n, len(a))
        ok = (a < b) & (block[a] != block[b])
        got = np.unique(np.concatenate([got, a[ok] * n + b[ok]]))
    got = rng.permutation(got)[:k]
    us.append(got // n)
    vs.append(got % n)
    return _symmetric_csr(n, np.concatenate(us), np.concatenate(vs))


def rmat(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         seed: int = 1, permute: bool = True, n: int | None = None) -> CSR:
    """R-MAT graph (Chakrabarti et al.): 2^scale vertices, edge_factor*2^scale
    generated edges, quadrant probabilities (a, b, c, 1-a-b-c), no noise.
    Symmetrised, self-loops and duplicates removed, unit weights; vertex ids
    optionally relabelled by a seeded random permutation.  If ``n`` is given the
    ids are folded into [0, n) after permutation (for non-power-of-two sizes)."""
    rng = _rng(seed)
    N = 1 << scale
    m = edge_factor * N
    ab, abc = a + b, a + b + c
    us, vs = [], []
    chunk = 1 << 22
    for s0 in range(0, m, chunk):
        k = min(chunk, m - s0)
        u = np.zeros(k, np.int64)
        v = np.zeros(k, np.int64)
        for _ in range(scale):
            r = rng.random(k, dtype=np.float32)
            bu = r >= ab                      # quadrants c or d: row bit 1
            bv = ((r >= a) & (r < ab)) | (r >= abc)  # quadrants b or d: column bit 1
            u = (u << 1) | bu
            v = (v << 1) | bv
        us.append(u)
        vs.append(v)
    u = np.concatenate(us)
    v = np.concatenate(vs)
    del us, vs
    if permute:
        perm = rng.permutation(N).astype(np.int64)
        u = perm[u]
        v = perm[v]
    nn = N
    if n is not None and n < N:
        u = u % n
        v = v % n
        nn = n
    return _symmetric_csr(nn, u, v)


def _assemble_device(N: int, key1, dev):
    """Symmetric CSR (rows sorted by neighbour id, unit weights) from the
    sorted unique undirected keys a*N+b (a < b) on a torch device: the rows'
    forward halves are key1, their backward halves the sorted mirrors; every
    entry's CSR position is its row offset plus its rank inside its own half
    of the row plus the number of entries of the other half of the row that
    precede it, found by binary search in the other sorted half."""
    import torch
    chunk = 1 << 26
    key2, _ = torch.sort((key1 % N) * N + key1 // N)
    bounds = torch.arange(N + 1, dtype=torch.int64, device=dev) * N
    h1 = torch.searchsorted(key1, bounds)
    h2 = torch.searchsorted(key2, bounds)
    deg = (h1[1:] - h1[:-1]) + (h2[1:] - h2[:-1])
    off = torch.zeros(N + 1, dtype=torch.int64, device=dev)
    off[1:] = torch.cumsum(deg, 0)
    nnz = int(off[-1].item())
    idx = torch.empty(nnz, dtype=torch.int32, device=dev)
    for mine, other, hm, ho in ((key1, key2, h1, h2), (key2, key1, h2, h1)):
        for s0 in range(0, mine.numel(), chunk):
            k = mine[s0:s0 + chunk]
            src = k // N
            rank = torch.arange(s0, s0 + k.numel(), dtype=torch.int64, device=dev) - hm[src]
            before = torch.searchsorted(other, k) - ho[src]
            idx[off[src] + rank + before] = (k % N).to(torch.int32)
            del k, src, rank, before
    del key2, h1, h2, bounds, deg
    w = torch.ones(nnz, dtype=torch.float32, device=dev)
    return off, idx, w


def rmat_device(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19, c: float = 0.19,
                seed: int = 1, device: str = "cuda", n: int | None = None):
    """The R-MAT graph of ``rmat`` (same model, symmetrised, self-loops and
    duplicates removed, unit weights, ids relabelled by a random permutation)
    drawn and assembled on a torch device, for sizes whose host assembly would
    take minutes (scale 26: ~1.9e9 directed entries).  Random numbers come from
    a ``torch.Generator`` seeded with ``seed``, so the graph differs from
    ``rmat``'s at the same seed.  With n < 2**scale the ids are folded modulo
    n (as ``rmat`` does).  Returns (n, off int64, idx int32, w float32) as
    device tensors, rows sorted by neighbour id."""
    import torch
    dev = torch.device(device)
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    N = 1 << scale
    m = edge_factor * N
    ab, abc = a + b, a + b + c
    perm = torch.randperm(N, generator=gen, device=dev)
    nn = n if (n is not None and n < N) else N
    chunk = 1 << 26
    keys = []
    for s0 in range(0, m, chunk):
        k = min(chunk, m - s0)
        u = torch.zeros(k, dtype=torch.int64, device=dev)
        v = torch.zeros(k, dtype=torch.int64, device=dev)
        for _ in range(scale):
            r = torch.rand(k, generator=gen, device=dev)
            u = (u << 1) | (r >= ab).to(torch.int64)
            v = (v << 1) | (((r >= a) & (r < ab)) | (r >= abc)).to(torch.int64)
        u = perm[u] % nn
        v = perm[v] % nn
        keep = u != v
        u, v = u[keep], v[keep]
        keys.append(torch.minimum(u, v) * nn + torch.maximum(u, v))
        del u, v, r, keep
    key1 = torch.unique(torch.cat(keys))          # sorted, a < b
    del keys, perm
    off, idx, w = _assemble_device(nn, key1, dev)
    return nn, off, idx, w


def planted_device(n: int, block: int = 64, deg_in: float = 6.3, deg_out: float = 4.0, seed: int = 1,
                   device: str = "cuda"):
    """Planted partition drawn on a torch device: vertices in consecutive
    blocks of `block` (ids then relabelled by a random permutation), about
    deg_in expected neighbours inside the block and deg_out outside per
    vertex: n*deg_in/2 intra-block and n*deg_out/2 inter-block vertex pairs
    drawn uniformly, repeats and self-loops dropped, unit weights.  Returns
    (n, off, idx, w) device tensors, rows sorted by neighbour id."""
    import torch
    dev = torch.device(device)
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    perm = torch.randperm(n, generator=gen, device=dev)
    m_in = int(round(n * deg_in / 2))
    m_out = int(round(n * deg_out / 2))
    u = torch.randint(0, n, (m_in,), generator=gen, device=dev)
    v = (u // block) * block + torch.randint(0, block, (m_in,), generator=gen, device=dev)
    v = torch.minimum(v, torch.full_like(v, n - 1))
    a = torch.randint(0, n, (m_out,), generator=gen, device=dev)
    b = torch.randint(0, n, (m_out,), generator=gen, device=dev)
    cross = (a // block) != (b // block)
    u = torch.cat([u, a[cross]])
    v = torch.cat([v, b[cross]])
    del a, b, cross
    u, v = perm[u], perm[v]
    keep = u != v
    u, v = u[keep], v[keep]
    key1 = torch.unique(torch.minimum(u, v) * n + torch.maximum(u, v))
    del u, v, keep, perm
    off, idx, w = _assemble_device(n, key1, dev)
    return n, off, idx, w


def grid2d(side: int = 4096, p_diag: float = 0.05, p_drop: float = 0.02, seed: int = 1) -> CSR:
    """Road-like graph: side x side 4-neighbour grid, each of the 2*(side-1)^2
    diagonals added with p_diag, then every edge dropped with p_drop."""
    rng = _rng(seed)
    ids = np.arange(side * side, dtype=np.int64).reshape(side, side)
    parts_u = [ids[:, :-1].ravel(), ids[:-1, :].ravel()]
    parts_v = [ids[:, 1:].ravel(), ids[1:, :].ravel()]
    d1u, d1v = ids[:-1, :-1].ravel(), ids[1:, 1:].ravel()
    d2u, d2v = ids[:-1, 1:].ravel(), ids[1:, :-1].ravel()
    k1 = rng.random(len(d1u)) < p_diag
    k2 = rng.random(len(d2u)) < p_diag
    parts_u += [d1u[k1], d2u[k2]]
    parts_v += [d1v[k1], d2v[k2]]
    u = np.concatenate(parts_u)
    v = np.concatenate(parts_v)
    keep = rng.random(len(u)) >= p_drop
    return _symmetric_csr(side * side, u[keep], v[keep])


def gnp(n: int, p: float, seed: int = 0, weights: str = "unit") -> CSR:
    """Erdos-Renyi G(n, p) for small tests; weights 'unit', 'int' (1..4) or 'float'."""
    rng = _rng(seed)
    iu, ju = np.triu_indices(n, k=1)
    keep = rng.random(len(iu)) < p
    u, v = iu[keep], ju[keep]
    if weights == "unit":
        w = np.ones(len(u), np.float32)
    elif weights == "int":
        w = rng.integers(1, 5, len(u)).astype(np.float32)
    else:
        w = (rng.random(len(u)) * 2.0 + 0.05).astype(np.float32)
    return from_edges(n, u, v, w)


def clique_ring(k: int, s: int) -> CSR:
    """k cliques of s vertices; clique t is joined to clique t+1 (mod k) by one edge."""
    us, vs = [], []
    for t in range(k):
        base = t * s
        iu, ju = np.triu_indices(s, k=1)
        us.append(base + iu)
        vs.append(base + ju)
        if k > 1 and not (k == 2 and t == 1):
            us.append(np.array([base + s - 1]))
            vs.append(np.array([((t + 1) % k) * s]))
    return from_edges(k * s, np.concatenate(us), np.concatenate(vs))


def disjoint_cliques(sizes) -> CSR:
    us, vs = [], []
    base = 0
    for s in sizes:
        iu, ju = np.triu_indices(s, k=1)
        us.append(base + iu)
        vs.append(base + ju)
        base += s
    return from_edges(base, np.concatenate(us), np.concatenate(vs))


def batch_count(nnz_directed: int, fraction: float) -> int:
    """Batch size in undirected updates: round(fraction * |E|), at least 1."""
    return max(1, int(round(fraction * nnz_directed)))


def _draw_updates(g: CSR, n_del: int, n_ins: int, rng: np.random.Generator):
    """n_del distinct existing undirected edges and n_ins distinct non-edge
    vertex pairs (no self-loops), each in a random orientation for inserts."""
    n = g.n
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(g.off))
    dst = g.idx.astype(np.int64)
    und = np.flatnonzero(src < dst)
    n_del = min(n_del, len(und))
    pick = np.empty(0, np.int64)
    while len(pick) < n_del:
        extra = rng.integers(0, len(und), 2 * (n_del - len(pick)) + 8)
        pick = np.unique(np.concatenate([pick, extra]))
    pick = rng.permutation(pick)[:n_del]
    e = und[pick]
    du, dv = src[e], dst[e]
    keys = src * n + dst  # globally sorted: rows ascend, entries ascend within rows
    got = np.empty(0, np.int64)
    while len(got) < n_ins and n > 1:
        k = 2 * (n_ins - len(got)) + 16
        a = rng.integers(0, n, k)
        b = rng.integers(0, n, k)
        lo, hi = np.minimum(a, b), np.maximum(a, b)
        ok = lo != hi
        cand = lo[ok] * n + hi[ok]
        pos = np.searchsorted(keys, cand)
        pos = np.minimum(pos, max(len(keys) - 1, 0))
        exists = (keys[pos] == cand) if len(keys) else np.zeros(len(cand), bool)
        cand = cand[~exists]
        merged = np.concatenate([got, cand])
        _, first = np.unique(merged, return_index=True)
        got = merged[np.sort(first)]
    got = got[:n_ins]
    iu, iv = got // n, got % n
    flip = rng.random(len(iu)) < 0.5
    iu, iv = np.where(flip, iv, iu), np.where(flip, iu, iv)
    return du, dv, iu, iv


def random_batch(g: CSR, size: int, ins_frac: float = 0.8, seed: int = 0,
                 weight: float = 1.0) -> UBatch:
    """Random batch (Sec. 5.1.4): round(ins_frac*size) insertions of uniformly
    random vertex pairs that are not edges (no self-loops, no repeats) and the
    rest deletions of distinct, uniformly chosen existing undirected edges."""
    n_ins = int(round(ins_frac * size))
    du, dv, iu, iv = _draw_updates(g, size - n_ins, n_ins, _rng(seed))
    return UBatch(du.astype(np.int32), dv.astype(np.int32), iu.astype(np.int32),
                  iv.astype(np.int32), np.full(len(iu), weight, np.float32))


def batch_stream(g: CSR, size: int, count: int, ins_frac: float = 0.8, seed: int = 0,
                 weight: float = 1.0) -> list:
    """`count` random batches of `size` updates each (split as in
    random_batch) that can be applied one after another starting from g:
    deletions are distinct edges of g across the whole stream, insertions
    distinct non-edges of g across the whole stream."""
    n_ins = int(round(ins_frac * size))
    n_del = size - n_ins
    du, dv, iu, iv = _draw_updates(g, n_del * count, n_ins * count, _rng(seed))
    out = []
    for k in range(count):
        d = slice(k * n_del, (k + 1) * n_del)
        i = slice(k * n_ins, (k + 1) * n_ins)
        out.append(UBatch(du[d].astype(np.int32), dv[d].astype(np.int32), iu[i].astype(np.int32),
                          iv[i].astype(np.int32), np.full(len(iu[i]), weight, np.float32)))
    return out


def batch_stream_device(n: int, off, idx, size, count: int, ins_frac: float = 0.8, seed: int = 0,
                        weight: float = 1.0) -> list:
    """The batch stream of ``batch_stream`` (Sec. 5.1.4: round(ins_frac*size)
    insertions of uniformly random non-edges, the rest deletions of uniformly
    chosen existing undirected edges, all distinct across the stream) drawn on
    the graph's torch device, for graphs whose host copy would be slow to
    search (RMAT scale 26).  off (int64, n+1) and idx (int32) are device
    tensors of a CSR with rows sorted by neighbour id.  Random numbers come
    from a ``torch.Generator`` seeded with ``seed``.  Returns a list of
    (del_u, del_v, ins_u, ins_v, ins_w) device tensors."""
    import torch
    dev = off.device
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    sizes = [int(size)] * count if np.isscalar(size) else [int(x) for x in size]
    count = len(sizes)
    ins = [int(round(ins_frac * x)) for x in sizes]
    dels = [x - y for x, y in zip(sizes, ins)]
    nnz = idx.numel()
    rows = torch.repeat_interleave(torch.arange(n, dtype=torch.int64, device=dev), off[1:] - off[:-1])
    keys = rows * n + idx.to(torch.int64)       # ascending: rows in order, sorted within rows
    del rows
    # deletions: an entry (u, v) with u < v names each undirected edge once;
    # entries are drawn uniformly, so each edge is equally likely
    need = sum(dels)
    picked = torch.empty(0, dtype=torch.int64, device=dev)
    while picked.numel() < need:
        e = torch.randint(0, nnz, (2 * (need - picked.numel()) + 64,), generator=gen, device=dev)
        k = keys[e]
        k = k[(k // n) < (k % n)]
        picked = torch.unique(torch.cat([picked, k]))
    picked = picked[torch.randperm(picked.numel(), generator=gen, device=dev)[:need]]
    # insertions: distinct unordered pairs that are not edges, random orientation
    need_i = sum(ins)
    got = torch.empty(0, dtype=torch.int64, device=dev)
    while got.numel() < need_i:
        k = 2 * (need_i - got.numel()) + 64
        a = torch.randint(0, n, (k,), generator=gen, device=dev)
        b = torch.randint(0, n, (k,), generator=gen, device=dev)
        lo, hi = torch.minimum(a, b), torch.maximum(a, b)
        ok = lo != hi
        cand = lo[ok] * n + hi[ok]
        pos = torch.clamp(torch.searchsorted(keys, cand), max=nnz - 1)
        cand = cand[keys[pos] != cand]
        got = torch.unique(torch.cat([got, cand]))
    got = got[torch.randperm(got.numel(), generator=gen, device=dev)[:need_i]]
    del keys
    flip = torch.rand(got.numel(), generator=gen, device=dev) < 0.5
    iu, iv = got // n, got % n
    iu, iv = torch.where(flip, iv, iu), torch.where(flip, iu, iv)
    du, dv = picked // n, picked % n
    out = []
    d0 = i0 = 0
    for j in range(count):
        d = slice(d0, d0 + dels[j])
        i = slice(i0, i0 + ins[j])
        d0 += dels[j]
        i0 += ins[j]
        out.append((du[d].to(torch.int32).contiguous(), dv[d].to(torch.int32).contiguous(),
                    iu[i].to(torch.int32).contiguous(), iv[i].to(torch.int32).contiguous(),
                    torch.full((ins[j],), weight, dtype=torch.float32, device=dev)))
    return out


def temporal_stream(gT: CSR, frac: float, count: int, preload: float = 0.9, ins_frac: float = 0.8,
                    seed: int = 0):
    """A synthetic stand-in for the paper's temporal graphs (Sec. 5.1.3,
    5.1.4): the undirected edges of gT get a seeded random order (their
    arrival times); the first `preload` fraction forms the initial graph, and
    then `count` consecutive batches of B = round(frac * |E_T|) updates follow
    (|E_T| = undirected edges of gT): round(ins_frac * B) insertions taken from
    the remaining edges in arrival order and the rest deletions of edges
    present at that point, chosen uniformly.  The stream stops early when the
    arrivals run out.  Returns (initial graph CSR, list of UBatch)."""
    rng = _rng(seed)
    src = np.repeat(np.arange(gT.n, dtype=np.int64), np.diff(gT.off))
    dst = gT.idx.astype(np.int64)
    und = np.flatnonzero(src < dst)
    und = und[rng.permutation(len(und))]
    eu, ev = src[und], dst[und]
    T = len(und)
    n0 = int(round(preload * T))
    B = max(1, int(round(frac * T)))
    n_ins = int(round(ins_frac * B))
    n_del = B - n_ins
    au = eu[:n0].copy()
    av = ev[:n0].copy()
    live = np.ones(len(au), bool)
    g0 = from_edges(gT.n, eu[:n0], ev[:n0])
    out = []
    nxt = n0
    for _ in range(count):
        if nxt + n_ins > T:
            break
        cand = np.flatnonzero(live)
        pick = cand[rng.choice(len(cand), size=min(n_del, len(cand)), replace=False)] if n_del else np.empty(0, np.int64)
        live[pick] = False
        du, dv = au[pick], av[pick]
        iu, iv = eu[nxt:nxt + n_ins], ev[nxt:nxt + n_ins]
        nxt += n_ins
        au = np.concatenate([au, iu])
        av = np.concatenate([av, iv])
        live = np.concatenate([live, np.ones(len(iu), bool)])
        out.append(UBatch(du.astype(np.int32), dv.astype(np.int32), iu.astype(np.int32), iv.astype(np.int32),
                          np.ones(len(iu), np.float32)))
    return g0, out
