"""Test-side helpers: brute force, exact modularity, partition utilities.

Nothing here implements a step of the method; these are independent checks.
"""
from fractions import Fraction
from functools import lru_cache

import numpy as np

import oracle


def as_og(g):
    """generator CSR -> oracle.Graph"""
    return oracle.as_graph(g.n, g.off, g.idx, g.w)


def edge_dict(g):
    d = {}
    for i in range(g.n):
        for e in range(int(g.off[i]), int(g.off[i + 1])):
            d[(i, int(g.idx[e]))] = float(g.w[e])
    return d


def dense_labels(C):
    _, inv = np.unique(np.asarray(C), return_inverse=True)
    return inv.astype(np.int32)


def canonical(C):
    """relabel by order of first occurrence"""
    C = np.asarray(C)
    out = np.empty(len(C), np.int64)
    seen = {}
    for i, c in enumerate(C):
        if c not in seen:
            seen[c] = len(seen)
        out[i] = seen[c]
    return out


def same_partition(a, b):
    return len(a) == len(b) and np.array_equal(canonical(a), canonical(b))


def q4_exact(g, C):
    """4 m^2 Q = M2 * sum_c sigma_c - sum_c S_c^2, exact (Fraction) - Newman's Q
    scaled by (2m)^2, with sigma over stored entries inside c and S_c = sum of K."""
    C = np.asarray(C)
    n = g.n
    src = np.repeat(np.arange(n), np.diff(g.off))
    w = [Fraction(float(x)) for x in g.w]
    M2 = sum(w, Fraction(0))
    sig = Fraction(0)
    S = {}
    for e in range(len(w)):
        ci = int(C[src[e]])
        if C[g.idx[e]] == ci:
            sig += w[e]
        S[ci] = S.get(ci, Fraction(0)) + w[e]
    return M2 * sig - sum((s * s for s in S.values()), Fraction(0))


@lru_cache(maxsize=None)
def rgs_partitions(n):
    """All set partitions of n items as restricted-growth strings (Bell(n) rows)."""
    out = []
    a = [0] * n

    def rec(i, m):
        if i == n:
            out.append(list(a))
            return
        for v in range(m + 2):
            a[i] = v
            rec(i + 1, max(m, v))

    if n == 0:
        return np.zeros((1, 0), np.int8)
    a[0] = 0
    rec(1, 0)
    return np.array(out, np.int8)


def brute_force_max_q4(g):
    """Maximum of 4m^2 Q over all set partitions (n <= 10); integer weights.
    Returns (max value as Fraction, list of optimal label arrays)."""
    n = g.n
    assert n <= 10
    P = rgs_partitions(n).astype(np.int64)
    src = np.repeat(np.arange(n), np.diff(g.off))
    dst = g.idx.astype(np.int64)
    w = g.w.astype(np.float64)
    assert np.all(w == np.round(w))
    K = np.zeros(n)
    np.add.at(K, src, w)
    M2 = K.sum()
    same = P[:, src] == P[:, dst]
    sig = same.astype(np.float64) @ w
    S2 = np.zeros(len(P))
    for c in range(n):
        Sc = (P == c).astype(np.float64) @ K
        S2 += Sc * Sc
    val = M2 * sig - S2          # exact: small integers in float64
    best = val.max()
    parts = [P[k] for k in np.flatnonzero(val == best)]
    return Fraction(int(best)), parts


def communities_connected(g, C):
    """Every community induces a connected subgraph (BFS)."""
    C = np.asarray(C)
    n = g.n
    seen = np.zeros(n, bool)
    for s in range(n):
        if seen[s]:
            continue
        c = C[s]
        stack = [s]
        seen[s] = True
        while stack:
            u = stack.pop()
            for e in range(int(g.off[u]), int(g.off[u + 1])):
                v = int(g.idx[e])
                if not seen[v] and C[v] == c:
                    seen[v] = True
                    stack.append(v)
        # any other unseen member of c means c is disconnected
    # second pass: each community must have been reached from a single start
    first = {}
    for s in range(n):
        first.setdefault(C[s], s)
    seen2 = np.zeros(n, bool)
    for c, s in first.items():
        stack = [s]
        seen2[s] = True
        while stack:
            u = stack.pop()
            for e in range(int(g.off[u]), int(g.off[u + 1])):
                v = int(g.idx[e])
                if not seen2[v] and C[v] == c:
                    seen2[v] = True
                    stack.append(v)
    return bool(seen2.all())
