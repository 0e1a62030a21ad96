"""Serial CPU oracle for dynamic Leiden (Static / ND / DS / DF).

TEST INFRASTRUCTURE ONLY.  This package is the plain reference the GPU library
is checked against.  Only the test-suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or call it; the product path
(the HIP library and its binding) never does.  It shares no code with the GPU
library: the C source in this directory is compiled on its own with gcc.

Each wrapper names the passage of Sahu, arXiv 2405.11658, that the C routine
follows; the readings taken where the paper is silent are stated in the C file.

Pins: tests/test_oracle_pins.py checks this oracle against brute-force maximum
modularity, closed forms, the textbook pairwise modularity, exact score
identities and invariants.  No function here is "parity unpinned".
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "leiden_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

MODE_ND, MODE_DS, MODE_DF = 1, 2, 3
MODES = {"nd": MODE_ND, "ds": MODE_DS, "df": MODE_DF}

OK, EINVAL, ENOMEM = 0, 1, 2
MAXP = 64


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no FMA contraction of decision scores)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
                               "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Params(ct.Structure):
    _fields_ = [("tau0", ct.c_double), ("tol_drop", ct.c_double), ("agg_tol", ct.c_double),
                ("max_iter", ct.c_int32), ("max_passes", ct.c_int32),
                ("sync_mode", ct.c_int32), ("refine_variant", ct.c_int32), ("nslices", ct.c_int32)]


class Stats(ct.Structure):
    _fields_ = [("passes", ct.c_int32),
                ("move_iters", ct.c_int32 * MAXP),
                ("refine_rounds", ct.c_int32 * MAXP),
                ("level_vertices", ct.c_int64 * MAXP),
                ("level_entries", ct.c_int64 * MAXP),
                ("communities", ct.c_int64 * MAXP),
                ("refined_vertices", ct.c_int64 * MAXP),
                ("affected", ct.c_int64),
                ("changed", ct.c_int64),
                ("moves_pass0", ct.c_int64)]

    def to_dict(self) -> dict:
        p = self.passes
        return {"passes": p, "move_iters": list(self.move_iters[:p]),
                "refine_rounds": list(self.refine_rounds[:p]),
                "level_vertices": list(self.level_vertices[:p]),
                "level_entries": list(self.level_entries[:p]),
                "communities": list(self.communities[:p]),
                "refined_vertices": list(self.refined_vertices[:p]),
                "affected": self.affected, "changed": self.changed,
                "moves_pass0": self.moves_pass0}


def make_params(sync: bool = False, tau0: float = 0.01, tol_drop: float = 10.0,
                agg_tol: float = 1.0, max_iter: int = 20, max_passes: int = 10,
                refine_variant: int = 0, nslices: int = 16) -> Params:
    """Defaults from Sec. 4.6 (tau0 = 0.01, drop 10, 20 iterations); passes 10;
    synchronous mode with 16 slices per sweep."""
    return Params(tau0, tol_drop, agg_tol, max_iter, max_passes, 1 if sync else 0, refine_variant,
                  nslices)


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=False)
        lib = ct.CDLL(_LIB)
        P = ct.c_void_p
        i64, i32, dbl = ct.c_int64, ct.c_int32, ct.c_double
        lib.or_modularity.argtypes = [i64, P, P, P, P, P]
        lib.or_aggregate.argtypes = [i64, P, P, P, P, i64, P, P, P, P]
        lib.or_apply_batch.argtypes = [i64, P, P, P, i64, P, P, i64, P, P, P, P, P, P, P]
        lib.or_mark.argtypes = [i32, i64, P, P, i64, P, P, i64, P, P, P, P, P, P, dbl, P, P, P]
        lib.or_update_weights.argtypes = [i64, P, P, P, i64, P, P, P, P, P, P, P]
        lib.or_update_weights.restype = None
        lib.or_core.argtypes = [i64, P, P, P, P, P, P, dbl, P, P, P, i32, P, P, P]
        lib.or_static.argtypes = [i64, P, P, P, P, P, P, P, P, P]
        lib.or_update.argtypes = [i32, i64, P, P, P, i64, P, P, P, i64, P, P, P, P, P, P, P, P, P, P, P, P]
        lib.or_best_move.argtypes = [i64, P, P, P, P, P, P, dbl, i32, P]
        lib.or_best_move.restype = i32
        lib.or_move_phase.argtypes = [i64, P, P, P, P, P, P, P, P, P, i32, dbl, dbl, i32, i32, P, P]
        lib.or_move_phase.restype = i32
        lib.or_subset_renumber.argtypes = [i64, P, P, P]
        lib.or_subset_renumber.restype = None
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ct.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _check(rc: int, what: str):
    if rc == EINVAL:
        raise ValueError(f"oracle {what}: invalid input")
    if rc != OK:
        raise MemoryError(f"oracle {what}: status {rc}")


@dataclass
class Graph:
    """CSR graph: int64 offsets, int32 neighbour ids, float32 weights."""
    n: int
    off: np.ndarray
    idx: np.ndarray
    w: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.off[-1])


def as_graph(n, off, idx, w) -> Graph:
    return Graph(int(n), _c(off, np.int64), _c(idx, np.int32), _c(w, np.float32))


def modularity(g: Graph, C) -> float:
    """Eq. 1 in FP64 (Sec. 3.2), sigma_c over stored entries, 0 when m = 0."""
    lib = _load()
    C = _c(C, np.int32)
    q = np.zeros(1, np.float64)
    _check(lib.or_modularity(g.n, _p(g.off), _p(g.idx), _p(g.w), _p(C), _p(q)), "modularity")
    return float(q[0])


def aggregate(g: Graph, C, ncomm: int) -> Graph:
    """Alg. leidenAggregate, canonical rows (ascending neighbour, FP64 sums rounded to float32)."""
    lib = _load()
    C = _c(C, np.int32)
    off = np.zeros(ncomm + 1, np.int64)
    idx = np.zeros(max(g.nnz, 1), np.int32)
    w = np.zeros(max(g.nnz, 1), np.float32)
    nnz = np.zeros(1, np.int64)
    _check(lib.or_aggregate(g.n, _p(g.off), _p(g.idx), _p(g.w), _p(C), ncomm,
                            _p(off), _p(idx), _p(w), _p(nnz)), "aggregate")
    k = int(nnz[0])
    return Graph(ncomm, off, idx[:k].copy(), w[:k].copy())


@dataclass
class Batch:
    """Undirected batch; each edge listed once (Sec. 5.1.4)."""
    del_u: np.ndarray
    del_v: np.ndarray
    ins_u: np.ndarray
    ins_v: np.ndarray
    ins_w: np.ndarray


def apply_batch(g: Graph, b: Batch):
    """G^t = G^{t-1} - deletions + insertions, both directions; returns (G^t, deleted weights)."""
    lib = _load()
    du, dv = _c(b.del_u, np.int32), _c(b.del_v, np.int32)
    iu, iv, iw = _c(b.ins_u, np.int32), _c(b.ins_v, np.int32), _c(b.ins_w, np.float32)
    cap = g.nnz + 2 * len(iu)
    off = np.zeros(g.n + 1, np.int64)
    idx = np.zeros(max(cap, 1), np.int32)
    w = np.zeros(max(cap, 1), np.float32)
    dw = np.zeros(max(len(du), 1), np.float32)
    _check(lib.or_apply_batch(g.n, _p(g.off), _p(g.idx), _p(g.w), len(du), _p(du), _p(dv),
                              len(iu), _p(iu), _p(iv), _p(iw), _p(off), _p(idx), _p(w), _p(dw)),
           "apply_batch")
    k = int(off[-1])
    return Graph(g.n, off, idx[:k].copy(), w[:k].copy()), dw[:len(du)].copy()


def mark(mode: str, gt: Graph, b: Batch, C_prev, K_prev, Sig_prev, M2_prev: float):
    """ND / DS / DF marking plus changedCommunities; returns (dV, in_range, dC) as uint8."""
    lib = _load()
    n = gt.n
    dV = np.zeros(max(n, 1), np.uint8)
    rng = np.zeros(max(n, 1), np.uint8)
    dC = np.zeros(max(n, 1), np.uint8)
    du, dv = _c(b.del_u, np.int32), _c(b.del_v, np.int32)
    iu, iv, iw = _c(b.ins_u, np.int32), _c(b.ins_v, np.int32), _c(b.ins_w, np.float32)
    C_prev, K_prev, Sig_prev = _c(C_prev, np.int32), _c(K_prev, np.float64), _c(Sig_prev, np.float64)
    _check(lib.or_mark(MODES[mode], n, _p(gt.off), _p(gt.idx), len(du), _p(du), _p(dv),
                       len(iu), _p(iu), _p(iv), _p(iw), _p(C_prev), _p(K_prev), _p(Sig_prev),
                       float(M2_prev), _p(dV), _p(rng), _p(dC)), "mark")
    return dV[:n].copy(), rng[:n].copy(), dC[:n].copy()


def update_weights(b: Batch, del_w, C_prev, K, Sig, M2: float):
    """Alg. updateWeights; returns new (K, Sigma, M2)."""
    lib = _load()
    K = _c(K, np.float64).copy()
    Sig = _c(Sig, np.float64).copy()
    m2 = np.array([M2], np.float64)
    du, dv, dw = _c(b.del_u, np.int32), _c(b.del_v, np.int32), _c(del_w, np.float32)
    iu, iv, iw = _c(b.ins_u, np.int32), _c(b.ins_v, np.int32), _c(b.ins_w, np.float32)
    C_prev = _c(C_prev, np.int32)
    lib.or_update_weights(len(du), _p(du), _p(dv), _p(dw), len(iu), _p(iu), _p(iv), _p(iw),
                          _p(C_prev), _p(K), _p(Sig), _p(m2))
    return K, Sig, float(m2[0])


def core(g: Graph, C_prev, K, Sig, M2: float, dV, in_range, dC0, track: bool,
         params: Params | None = None):
    """Alg. leiden (the pass loop) on level-0 graph g; returns (membership, stats dict)."""
    lib = _load()
    params = params or make_params()
    n = g.n
    out = np.zeros(max(n, 1), np.int32)
    st = Stats()
    args = [_c(C_prev, np.int32), _c(K, np.float64), _c(Sig, np.float64)]
    flags = [_c(dV, np.uint8), _c(in_range, np.uint8), _c(dC0, np.uint8)]
    _check(lib.or_core(n, _p(g.off), _p(g.idx), _p(g.w), _p(args[0]), _p(args[1]), _p(args[2]),
                       float(M2), _p(flags[0]), _p(flags[1]), _p(flags[2]), 1 if track else 0,
                       ct.byref(params), _p(out), ct.byref(st)), "core")
    return out[:n].copy(), st.to_dict()


@dataclass
class State:
    """Carried state between batches: graph, membership, K, Sigma, M2 (Sec. 5.1.5)."""
    g: Graph
    C: np.ndarray
    K: np.ndarray
    Sig: np.ndarray
    M2: float


def static(g: Graph, params: Params | None = None):
    """Static Leiden from singletons; returns (State, stats)."""
    lib = _load()
    params = params or make_params()
    n = g.n
    C = np.zeros(max(n, 1), np.int32)
    K = np.zeros(max(n, 1), np.float64)
    Sig = np.zeros(max(n, 1), np.float64)
    m2 = np.zeros(1, np.float64)
    st = Stats()
    _check(lib.or_static(n, _p(g.off), _p(g.idx), _p(g.w), ct.byref(params), _p(C), _p(K), _p(Sig),
                         _p(m2), ct.byref(st)), "static")
    return State(g, C[:n].copy(), K[:n].copy(), Sig[:n].copy(), float(m2[0])), st.to_dict()


def update(state: State, b: Batch, mode: str, params: Params | None = None):
    """Apply the batch, then ND/DS/DF Leiden (Alg. naiveDynamic / deltaScreening /
    dynamicFrontier).  Returns (new State, dV, dC, stats)."""
    lib = _load()
    params = params or make_params()
    gt, dw = apply_batch(state.g, b)
    n = gt.n
    K = state.K.copy()
    Sig = state.Sig.copy()
    m2 = np.array([state.M2], np.float64)
    C = np.zeros(max(n, 1), np.int32)
    dV = np.zeros(max(n, 1), np.uint8)
    dC = np.zeros(max(n, 1), np.uint8)
    du, dv = _c(b.del_u, np.int32), _c(b.del_v, np.int32)
    iu, iv, iw = _c(b.ins_u, np.int32), _c(b.ins_v, np.int32), _c(b.ins_w, np.float32)
    st = Stats()
    _check(lib.or_update(MODES[mode], n, _p(gt.off), _p(gt.idx), _p(gt.w), len(du), _p(du), _p(dv),
                         _p(dw), len(iu), _p(iu), _p(iv), _p(iw), _p(state.C), _p(K), _p(Sig),
                         _p(m2), ct.byref(params), _p(C), _p(dV), _p(dC), ct.byref(st)), "update")
    new = State(gt, C[:n].copy(), K, Sig, float(m2[0]))
    return new, dV[:n].copy(), dC[:n].copy(), st.to_dict()


def best_move(g: Graph, C, K, Sig, M2: float, i: int):
    """One local-moving decision (Alg. leidenMove body, Eq. 2); returns (target or -1, g)."""
    lib = _load()
    C, K, Sig = _c(C, np.int32), _c(K, np.float64), _c(Sig, np.float64)
    gout = np.zeros(1, np.float64)
    c = lib.or_best_move(g.n, _p(g.off), _p(g.idx), _p(g.w), _p(C), _p(K), _p(Sig), float(M2),
                         int(i), _p(gout))
    return int(c), float(gout[0])


def move_phase(g: Graph, C, K, Sig, M2: float, dC, U, rng, track: bool, tau: float = 0.01,
               max_iter: int = 20, sync: bool = False, nslices: int = 16):
    """One local-moving phase (Alg. leidenMove); returns (iterations, C, Sig, dC, U, moves,
    total gain in units of 2m^2)."""
    lib = _load()
    C = _c(C, np.int32).copy(); Sig = _c(Sig, np.float64).copy()
    dC = _c(dC, np.uint8).copy(); U = _c(U, np.uint8).copy()
    K = _c(K, np.float64); rng = _c(rng, np.uint8)
    nm = np.zeros(1, np.int64)
    gain = np.zeros(1, np.float64)
    l = lib.or_move_phase(g.n, _p(g.off), _p(g.idx), _p(g.w), _p(C), _p(K), _p(Sig), _p(dC), _p(U),
                          _p(rng), 1 if track else 0, float(M2), float(tau), int(max_iter),
                          int(nslices) if sync else 0, _p(nm), _p(gain))
    return int(l), C, Sig, dC, U, int(nm[0]), float(gain[0])


def subset_renumber(C, Sig, dC):
    """Alg. leidenSubsetRenumber (representative = smallest member id)."""
    lib = _load()
    C = _c(C, np.int32).copy(); Sig = _c(Sig, np.float64).copy(); dC = _c(dC, np.uint8).copy()
    lib.or_subset_renumber(len(C), _p(C), _p(Sig), _p(dC))
    return C, Sig, dC
