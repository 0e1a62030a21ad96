"""Thin Python binding of the HIP library ``libleiden_hip.so`` (C ABI in
``include/leiden.h``).  Argument marshalling only: every step of the method
runs in the library's kernels.  Tensors are torch tensors on the current HIP
device; the current torch stream is passed to every call.

The functions carry the C names.  Loading fails loudly when the library has
not been built (run ``python paper_2405_11658_amd/build.py``) - there is no
CPU fallback.
"""
from __future__ import annotations

import ctypes as ct
import os
import threading
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libleiden_hip.so")

OK, EINVAL, ENOMEM, ESTATE, EHIP = 0, 1, 2, 3, 4
ND, DS, DF = 1, 2, 3
MODES = {"nd": ND, "ds": DS, "df": DF}
MAX_PASSES = 64


class LeidenError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


# kernels timed with leiden_params.profile = 1, in LEIDEN_PROF_* order
PROF_KERNELS = ("hub_gather", "agg_merge", "mod_scan", "batch_merge", "move_sweep", "refine_sweep")
PROF_N = len(PROF_KERNELS)


class leiden_params(ct.Structure):
    _fields_ = [("tau0", ct.c_double), ("tol_drop", ct.c_double), ("agg_tol", ct.c_double),
                ("max_iter", ct.c_int32), ("max_passes", ct.c_int32),
                ("sync_mode", ct.c_int32), ("refine_variant", ct.c_int32), ("nslices", ct.c_int32),
                ("profile", ct.c_int32), ("async_waves", ct.c_int32),
                ("hub_slices", ct.c_int32), ("verts_per_wave", ct.c_int32),
                ("verts_per_wave_upper", ct.c_int32), ("hub_degree", ct.c_int32), ("trim", ct.c_int32)]


class leiden_stats(ct.Structure):
    _fields_ = [("passes", ct.c_int32),
                ("move_iters", ct.c_int32 * MAX_PASSES),
                ("refine_rounds", ct.c_int32 * MAX_PASSES),
                ("level_vertices", ct.c_int64 * MAX_PASSES),
                ("level_entries", ct.c_int64 * MAX_PASSES),
                ("communities", ct.c_int64 * MAX_PASSES),
                ("refined_vertices", ct.c_int64 * MAX_PASSES),
                ("affected", ct.c_int64), ("changed", ct.c_int64), ("moves_pass0", ct.c_int64),
                ("ms_total", ct.c_double), ("ms_apply", ct.c_double), ("ms_mark", ct.c_double),
                ("ms_move", ct.c_double), ("ms_refine", ct.c_double), ("ms_aggregate", ct.c_double),
                ("ms_other", ct.c_double),
                ("prof_launches", ct.c_int64 * PROF_N), ("prof_ms", ct.c_double * PROF_N),
                ("prof_entries", ct.c_int64 * PROF_N), ("prof_vertices", ct.c_int64 * PROF_N),
                ("pass_move_ms", ct.c_double * MAX_PASSES), ("pass_refine_ms", ct.c_double * MAX_PASSES),
                ("pass_agg_ms", ct.c_double * MAX_PASSES)]

    def to_dict(self) -> dict:
        p = self.passes
        d = {"passes": p, "move_iters": list(self.move_iters[:p]),
             "refine_rounds": list(self.refine_rounds[:p]),
             "level_vertices": list(self.level_vertices[:p]),
             "level_entries": list(self.level_entries[:p]),
             "communities": list(self.communities[:p]),
             "refined_vertices": list(self.refined_vertices[:p]),
             "affected": self.affected, "changed": self.changed, "moves_pass0": self.moves_pass0,
             "pass_move_ms": list(self.pass_move_ms[:p]), "pass_refine_ms": list(self.pass_refine_ms[:p]),
             "pass_agg_ms": list(self.pass_agg_ms[:p])}
        for k in ("ms_total", "ms_apply", "ms_mark", "ms_move", "ms_refine", "ms_aggregate", "ms_other"):
            d[k] = getattr(self, k)
        d["prof"] = {name: {"launches": self.prof_launches[k], "ms": self.prof_ms[k],
                            "entries": self.prof_entries[k], "vertices": self.prof_vertices[k]}
                     for k, name in enumerate(PROF_KERNELS)}
        return d


class leiden_batch(ct.Structure):
    _fields_ = [("n_del", ct.c_int64), ("del_u", ct.c_void_p), ("del_v", ct.c_void_p),
                ("n_ins", ct.c_int64), ("ins_u", ct.c_void_p), ("ins_v", ct.c_void_p),
                ("ins_w", ct.c_void_p)]


class leiden_trace(ct.Structure):
    _fields_ = [("affected", ct.c_void_p), ("in_range", ct.c_void_p), ("changed", ct.c_void_p)]


_ALLOC_FN = ct.CFUNCTYPE(ct.c_void_p, ct.c_void_p, ct.c_size_t, ct.c_void_p)
_RELEASE_FN = ct.CFUNCTYPE(None, ct.c_void_p, ct.c_void_p, ct.c_size_t, ct.c_void_p)


class leiden_allocator(ct.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("release", _RELEASE_FN), ("ctx", ct.c_void_p)]


class TorchAllocator:
    """leiden_allocator backed by torch's caching allocator.  Blocks are taken
    on (and returned to) the device's default stream, whatever stream the
    library names, because the library's own worker streams may be gone by
    the time a block is released: a block handed to work on another stream
    is ordered after the default stream's pending work (that stream waits for
    an event), and a block released from another stream returns to the pool
    only after the work enqueued there (the default stream waits for it)."""

    def __init__(self):
        self._alloc_cb = _ALLOC_FN(self._alloc)
        self._release_cb = _RELEASE_FN(self._release)
        self.c = leiden_allocator(self._alloc_cb, self._release_cb, None)

    def _alloc(self, ctx, nbytes, stream):
        try:
            dev = torch.cuda.current_device()
            home = torch.cuda.default_stream(dev)
            p = torch.cuda.caching_allocator_alloc(int(nbytes), dev, home)
            if stream and stream != home.cuda_stream:
                ev = torch.cuda.Event()
                ev.record(home)
                torch.cuda.ExternalStream(stream).wait_event(ev)
        except RuntimeError:
            return None
        return p

    def _release(self, ctx, ptr, nbytes, stream):
        dev = torch.cuda.current_device()
        home = torch.cuda.default_stream(dev)
        if stream and stream != home.cuda_stream:
            ev = torch.cuda.Event()
            ev.record(torch.cuda.ExternalStream(stream))
            home.wait_event(ev)
        torch.cuda.caching_allocator_delete(ptr)


_torch_alloc = None


def torch_allocator() -> TorchAllocator:
    global _torch_alloc
    if _torch_alloc is None:
        _torch_alloc = TorchAllocator()
    return _torch_alloc


_lib = None


def load() -> ct.CDLL:
    """Load libleiden_hip.so; raises if it is missing (no fallback path exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"HIP library not built: {LIB_PATH} (run paper_2405_11658_amd/build.py)")
    lib = ct.CDLL(LIB_PATH)
    P, i64, i32, dbl = ct.c_void_p, ct.c_int64, ct.c_int32, ct.c_double
    sig = {
        "leiden_default_params": (None, [P]),
        "leiden_create": (i32, [i64, i64, P, P, P, P, P, P, P]),
        "leiden_mark_affected": (i32, [P, P, i32, P, P, P, P]),
        "leiden_fleet_create": (i32, [i32, P, P, P, P, P, P, P, P, P]),
        "leiden_fleet_run": (i32, [P, i32, P, P, P, P, P, P, P, P, P]),
        "leiden_fleet_get_graph": (i32, [P, i32, P, P, P, P, P]),
        "leiden_fleet_get_state": (i32, [P, i32, P, P, P, P, P]),
        "leiden_fleet_set_variant": (i32, [P, i32]),
        "leiden_fleet_variant_info": (i32, [i32, P, P]),
        "leiden_fleet_count": (i32, [P]),
        "leiden_fleet_last_error": (ct.c_char_p, [P]),
        "leiden_fleet_destroy": (i32, [P]),
        "leiden_update_bytes": (i32, [P, i64, i64, P]),
        "leiden_destroy": (i32, [P]),
        "leiden_set_params": (i32, [P, P]),
        "leiden_static": (i32, [P, P, P, P, P]),
        "leiden_update": (i32, [P, P, i32, P, P, P, P, P]),
        "leiden_update_many": (i32, [P, P, P, i32, P, P, P, P, i32, P]),
        "leiden_server_create": (i32, [i32, i64, P]),
        "leiden_server_submit": (i32, [P, P, P, i32, P, P]),
        "leiden_server_wait": (i32, [P, i64, P, P, P, P, P]),
        "leiden_server_submit_fleet": (i32, [P, P, i32, P, i32, P, P]),
        "leiden_server_destroy": (i32, [P]),
        "leiden_modularity": (i32, [i64, P, P, P, P, P, P]),
        "leiden_aggregate": (i32, [i64, P, P, P, P, i64, P, P, P, P, P]),
        "leiden_get_graph": (i32, [P, P, P, P, P, P]),
        "leiden_get_state": (i32, [P, P, P, P, P, P]),
        "leiden_set_state": (i32, [P, P, P]),
        "leiden_num_vertices": (i64, [P]),
        "leiden_num_entries": (i64, [P]),
        "leiden_strerror": (ct.c_char_p, [i32]),
        "leiden_last_error": (ct.c_char_p, [P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _stream():
    return ct.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: torch.Tensor | None):
    return ct.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else ct.c_void_p(0)


def _dev(x, dtype) -> torch.Tensor:
    if isinstance(x, torch.Tensor):
        return x.to(device="cuda", dtype=dtype).contiguous()
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def _check(st: int, handle=None, what: str = ""):
    if st != OK:
        lib = load()
        msg = lib.leiden_last_error(handle).decode() if handle else ""
        if not msg:
            msg = lib.leiden_strerror(st).decode()
        raise LeidenError(st, f"{what}: {msg}")


def leiden_default_params(**overrides) -> leiden_params:
    p = leiden_params()
    load().leiden_default_params(ct.byref(p))
    for k, v in overrides.items():
        setattr(p, k, v)
    return p


@dataclass
class Handle:
    ptr: ct.c_void_p
    n: int

    def __del__(self):
        if self.ptr and _lib is not None:
            _lib.leiden_destroy(self.ptr)
            self.ptr = None


def leiden_create(off, idx, w, params: leiden_params | None = None, allocator="torch") -> Handle:
    """Copy a CSR graph (int64 offsets, int32 ids, float32 weights) into a new handle.
    allocator: "torch" (torch's caching allocator, the default) or None (the
    library's own stream-ordered allocation)."""
    lib = load()
    off = _dev(off, torch.int64)
    idx = _dev(idx, torch.int32)
    w = _dev(w, torch.float32)
    n = off.numel() - 1
    out = ct.c_void_p()
    al = ct.byref(torch_allocator().c) if allocator == "torch" else None
    st = lib.leiden_create(n, idx.numel(), _ptr(off), _ptr(idx), _ptr(w),
                           ct.byref(params) if params is not None else None, al, _stream(), ct.byref(out))
    _check(st, None, "leiden_create")
    return Handle(out, n)


def leiden_destroy(h: Handle):
    if h.ptr:
        _check(load().leiden_destroy(h.ptr), None, "leiden_destroy")
        h.ptr = None


def leiden_set_params(h: Handle, params: leiden_params):
    _check(load().leiden_set_params(h.ptr, ct.byref(params)), h.ptr, "leiden_set_params")


def leiden_static(h: Handle, want_q: bool = True):
    """Static Leiden.  Returns (membership int32 tensor, modularity or None, stats dict)."""
    lib = load()
    out = torch.empty(h.n, dtype=torch.int32, device="cuda")
    q = ct.c_double(0.0)
    st = leiden_stats()
    _check(lib.leiden_static(h.ptr, _ptr(out), ct.byref(q) if want_q else None, ct.byref(st), _stream()),
           h.ptr, "leiden_static")
    return out, (q.value if want_q else None), st.to_dict()


def make_batch(del_u, del_v, ins_u, ins_v, ins_w):
    """Device tensors of an undirected batch (each edge once)."""
    return (_dev(del_u, torch.int32), _dev(del_v, torch.int32), _dev(ins_u, torch.int32),
            _dev(ins_v, torch.int32), _dev(ins_w, torch.float32))


def leiden_update(h: Handle, batch, mode, want_q: bool = True, trace: bool = False):
    """Apply a batch and run ND/DS/DF Leiden.  batch = (del_u, del_v, ins_u, ins_v, ins_w)
    device tensors (see make_batch).  Returns (membership, q, stats, trace dict or None)."""
    lib = load()
    if isinstance(mode, str):
        mode = MODES[mode]
    du, dv, iu, iv, iw = batch
    b = leiden_batch(du.numel(), _ptr(du), _ptr(dv), iu.numel(), _ptr(iu), _ptr(iv), _ptr(iw))
    out = torch.empty(h.n, dtype=torch.int32, device="cuda")
    q = ct.c_double(0.0)
    st = leiden_stats()
    tr = None
    trs = None
    if trace:
        tr = {k: torch.zeros(max(h.n, 1), dtype=torch.uint8, device="cuda")
              for k in ("affected", "in_range", "changed")}
        trs = leiden_trace(_ptr(tr["affected"]), _ptr(tr["in_range"]), _ptr(tr["changed"]))
    _check(lib.leiden_update(h.ptr, ct.byref(b), int(mode), _ptr(out), ct.byref(q) if want_q else None,
                             ct.byref(st), ct.byref(trs) if trs is not None else None, _stream()),
           h.ptr, "leiden_update")
    if tr is not None:
        tr = {k: v[:h.n] for k, v in tr.items()}
    return out, (q.value if want_q else None), st.to_dict(), tr


def _cbatch(batch):
    du, dv, iu, iv, iw = batch
    return leiden_batch(du.numel(), _ptr(du), _ptr(dv), iu.numel(), _ptr(iu), _ptr(iv), _ptr(iw))


def leiden_mark_affected(h: Handle, batch, mode):
    """Flags leiden_update would compute for this batch, without changing the
    handle: dict of uint8 tensors affected / in_range / changed (n each)."""
    if isinstance(mode, str):
        mode = MODES[mode]
    tr = {k: torch.zeros(max(h.n, 1), dtype=torch.uint8, device="cuda") for k in ("affected", "in_range", "changed")}
    b = _cbatch(batch)
    _check(load().leiden_mark_affected(h.ptr, ct.byref(b), int(mode), _ptr(tr["affected"]), _ptr(tr["in_range"]),
                                       _ptr(tr["changed"]), _stream()), h.ptr, "leiden_mark_affected")
    return {k: v[:h.n] for k, v in tr.items()}


def leiden_update_bytes(h: Handle, n_del: int, n_ins: int) -> int:
    out = ct.c_int64(0)
    _check(load().leiden_update_bytes(h.ptr, int(n_del), int(n_ins), ct.byref(out)), h.ptr, "leiden_update_bytes")
    return out.value


def leiden_update_many(handles, batches, modes, want_q: bool = True, max_parallel: int = 0):
    """Batched updates of distinct handles (run concurrently by the library).
    Returns a list of (membership, q or None, stats dict, status) per handle;
    raises LeidenError only for a malformed call (nothing ran)."""
    lib = load()
    k = len(handles)
    H = (ct.c_void_p * k)(*[h.ptr for h in handles])
    B = (leiden_batch * k)()
    keep = []
    for j, (du, dv, iu, iv, iw) in enumerate(batches):
        B[j] = leiden_batch(du.numel(), _ptr(du), _ptr(dv), iu.numel(), _ptr(iu), _ptr(iv), _ptr(iw))
        keep.append((du, dv, iu, iv, iw))
    M = (ct.c_int32 * k)(*[MODES[m] if isinstance(m, str) else int(m) for m in modes])
    outs = [torch.empty(h.n, dtype=torch.int32, device="cuda") for h in handles]
    O = (ct.c_void_p * k)(*[_ptr(o) for o in outs])
    Q = (ct.c_double * k)()
    S = (leiden_stats * k)()
    ST = (ct.c_int32 * k)()
    st = lib.leiden_update_many(H, B, M, k, O, Q if want_q else None, S, ST, max_parallel, _stream())
    if st != OK and all(x == OK for x in ST):
        raise LeidenError(st, "leiden_update_many")
    return [(outs[j], (Q[j] if want_q else None), S[j].to_dict(), int(ST[j])) for j in range(k)]


class Server:
    """leiden_server_*: queued update requests over resident handles."""

    def __init__(self, slots: int = 4, memory_budget: int = 0):
        self.ptr = ct.c_void_p()
        _check(load().leiden_server_create(slots, memory_budget, ct.byref(self.ptr)), None,
               "leiden_server_create")
        self._pending = {}

    def submit(self, h: Handle, batch, mode) -> int:
        """Queue an update of handle h; returns the request id."""
        if isinstance(mode, str):
            mode = MODES[mode]
        du, dv, iu, iv, iw = batch
        b = leiden_batch(du.numel(), _ptr(du), _ptr(dv), iu.numel(), _ptr(iu), _ptr(iv), _ptr(iw))
        out = torch.empty(h.n, dtype=torch.int32, device="cuda")
        rid = ct.c_int64()
        _check(load().leiden_server_submit(self.ptr, h.ptr, ct.byref(b), int(mode), _ptr(out), ct.byref(rid)),
               None, "leiden_server_submit")
        self._pending[rid.value] = (out, b, batch, h)  # keep buffers alive until wait
        return rid.value

    def submit_fleet(self, fleet, graph: int, batch, mode) -> int:
        """Queue a job on graph `graph` of a Fleet (mode "static" with batch
        None, or "nd" / "ds" / "df"); returns the request id."""
        m = FLEET_STATIC if mode == "static" else MODES[mode] if isinstance(mode, str) else int(mode)
        b = _cbatch(batch) if batch is not None else None
        out = torch.empty(max(fleet.n[graph], 1), dtype=torch.int32, device="cuda")
        rid = ct.c_int64()
        _check(load().leiden_server_submit_fleet(self.ptr, fleet.ptr, int(graph), ct.byref(b) if b is not None else None,
                                                 int(m), _ptr(out), ct.byref(rid)), None, "leiden_server_submit_fleet")
        self._pending[rid.value] = (out, b, batch, fleet)
        return rid.value

    def wait(self, rid: int):
        """Block until request rid is done: (status, membership, q, stats, latency_ms, service_ms)."""
        st = ct.c_int32()
        q = ct.c_double()
        s = leiden_stats()
        lat = ct.c_double()
        svc = ct.c_double()
        _check(load().leiden_server_wait(self.ptr, rid, ct.byref(st), ct.byref(q), ct.byref(s), ct.byref(lat),
                                         ct.byref(svc)), None, "leiden_server_wait")
        out, _, _, _ = self._pending.pop(rid)
        return st.value, out, q.value, s.to_dict(), lat.value, svc.value

    def close(self):
        if self.ptr:
            load().leiden_server_destroy(self.ptr)
            self.ptr = None
            self._pending.clear()

    def __del__(self):
        if self.ptr and _lib is not None:
            _lib.leiden_server_destroy(self.ptr)
            self.ptr = None


def leiden_modularity(off, idx, w, membership) -> float:
    lib = load()
    off = _dev(off, torch.int64)
    idx = _dev(idx, torch.int32)
    w = _dev(w, torch.float32)
    C = _dev(membership, torch.int32)
    q = ct.c_double(0.0)
    _check(lib.leiden_modularity(off.numel() - 1, _ptr(off), _ptr(idx), _ptr(w), _ptr(C), ct.byref(q),
                                 _stream()), None, "leiden_modularity")
    return q.value


def leiden_aggregate(off, idx, w, membership, ncomm: int):
    """Super-vertex CSR (rows compacted and sorted by neighbour id)."""
    lib = load()
    off = _dev(off, torch.int64)
    idx = _dev(idx, torch.int32)
    w = _dev(w, torch.float32)
    C = _dev(membership, torch.int32)
    cap = max(idx.numel(), 1)
    ooff = torch.zeros(ncomm + 1, dtype=torch.int64, device="cuda")
    oidx = torch.empty(cap, dtype=torch.int32, device="cuda")
    ow = torch.empty(cap, dtype=torch.float32, device="cuda")
    nnz = ct.c_int64(0)
    _check(lib.leiden_aggregate(off.numel() - 1, _ptr(off), _ptr(idx), _ptr(w), _ptr(C), ncomm, _ptr(ooff),
                                _ptr(oidx), _ptr(ow), ct.byref(nnz), _stream()), None, "leiden_aggregate")
    k = nnz.value
    return ooff, oidx[:k], ow[:k]


def leiden_get_graph(h: Handle):
    lib = load()
    nnz = ct.c_int64(0)
    _check(lib.leiden_get_graph(h.ptr, None, None, None, ct.byref(nnz), _stream()), h.ptr, "leiden_get_graph")
    off = torch.empty(h.n + 1, dtype=torch.int64, device="cuda")
    idx = torch.empty(max(nnz.value, 1), dtype=torch.int32, device="cuda")
    w = torch.empty(max(nnz.value, 1), dtype=torch.float32, device="cuda")
    _check(lib.leiden_get_graph(h.ptr, _ptr(off), _ptr(idx), _ptr(w), ct.byref(nnz), _stream()), h.ptr,
           "leiden_get_graph")
    return off, idx[:nnz.value], w[:nnz.value]


def leiden_get_state(h: Handle):
    lib = load()
    C = torch.empty(max(h.n, 1), dtype=torch.int32, device="cuda")
    K = torch.empty(max(h.n, 1), dtype=torch.float64, device="cuda")
    S = torch.empty(max(h.n, 1), dtype=torch.float64, device="cuda")
    m2 = ct.c_double(0.0)
    _check(lib.leiden_get_state(h.ptr, _ptr(C), _ptr(K), _ptr(S), ct.byref(m2), _stream()), h.ptr,
           "leiden_get_state")
    return C[:h.n], K[:h.n], S[:h.n], m2.value


def leiden_set_state(h: Handle, membership):
    C = _dev(membership, torch.int32)
    _check(load().leiden_set_state(h.ptr, _ptr(C), _stream()), h.ptr, "leiden_set_state")


def leiden_num_vertices(h: Handle) -> int:
    return int(load().leiden_num_vertices(h.ptr))


def leiden_num_entries(h: Handle) -> int:
    return int(load().leiden_num_entries(h.ptr))


FLEET_STATIC = 0
FLEET_VARIANTS = 6


def fleet_variant_info(v: int):
    """(wavefronts per workgroup, LDS table slots) of fleet launch variant v."""
    w, sl = ct.c_int32(), ct.c_int32()
    _check(load().leiden_fleet_variant_info(int(v), ct.byref(w), ct.byref(sl)), None, "leiden_fleet_variant_info")
    return w.value, sl.value


class Fleet:
    """leiden_fleet_*: many small graphs updated together, one persistent
    launch per run (see include/leiden.h)."""

    def __init__(self, graphs, params: leiden_params | None = None, allocator="torch"):
        lib = load()
        self.ptr = ct.c_void_p()
        self._dev = []
        ns, nnzs, offs, idxs, ws = [], [], [], [], []
        for off, idx, w in graphs:
            off = _dev(off, torch.int64)
            idx = _dev(idx, torch.int32)
            w = _dev(w, torch.float32)
            self._dev.append((off, idx, w))
            ns.append(off.numel() - 1)
            nnzs.append(idx.numel())
        k = len(ns)
        self.n = ns
        N = (ct.c_int64 * k)(*ns)
        Z = (ct.c_int64 * k)(*nnzs)
        O = (ct.c_void_p * k)(*[_ptr(d[0]).value for d in self._dev])
        I = (ct.c_void_p * k)(*[_ptr(d[1]).value for d in self._dev])
        W = (ct.c_void_p * k)(*[_ptr(d[2]).value for d in self._dev])
        al = ct.byref(torch_allocator().c) if allocator == "torch" else None
        st = lib.leiden_fleet_create(k, N, Z, O, I, W, ct.byref(params) if params is not None else None, al,
                                     _stream(), ct.byref(self.ptr))
        self._dev = None
        if st != OK:
            raise LeidenError(st, "leiden_fleet_create")

    def _err(self, st, what):
        if st != OK:
            msg = load().leiden_fleet_last_error(self.ptr).decode() or load().leiden_strerror(st).decode()
            raise LeidenError(st, f"{what}: {msg}")

    def set_variant(self, v: int):
        self._err(load().leiden_fleet_set_variant(self.ptr, int(v)), "leiden_fleet_set_variant")

    def run(self, jobs, want_membership: bool = True):
        """jobs: list of (graph index, mode, batch) with mode "static" / "nd" /
        "ds" / "df" (batch None for static, else make_batch tensors).  One
        launch.  Returns (list of (membership or None, q, status, stats dict),
        launch ms)."""
        lib = load()
        k = len(jobs)
        G = (ct.c_int32 * k)(*[int(j[0]) for j in jobs])
        M = (ct.c_int32 * k)(*[FLEET_STATIC if j[1] == "static" else MODES[j[1]] if isinstance(j[1], str) else int(j[1])
                               for j in jobs])
        B = (leiden_batch * k)()
        keep = []
        for q, (_, mode, batch) in enumerate(jobs):
            if batch is not None:
                B[q] = _cbatch(batch)
                keep.append(batch)
        outs = [torch.empty(max(self.n[int(j[0])], 1), dtype=torch.int32, device="cuda") if want_membership else None
                for j in jobs]
        O = (ct.c_void_p * k)(*[_ptr(o).value if o is not None else None for o in outs])
        Q = (ct.c_double * k)()
        ST = (ct.c_int32 * k)()
        S = (leiden_stats * k)()
        ms = ct.c_double(0.0)
        st = lib.leiden_fleet_run(self.ptr, k, G, M, B, O if want_membership else None, Q, ST, S, ct.byref(ms),
                                  _stream())
        if st != OK and all(x == OK for x in ST):
            self._err(st, "leiden_fleet_run")
        res = []
        for q in range(k):
            n = self.n[int(jobs[q][0])]
            res.append(((outs[q][:n] if outs[q] is not None else None), Q[q], int(ST[q]), S[q].to_dict()))
        return res, ms.value

    def get_graph(self, k: int):
        lib = load()
        nnz = ct.c_int64(0)
        self._err(lib.leiden_fleet_get_graph(self.ptr, k, None, None, None, ct.byref(nnz), _stream()),
                  "leiden_fleet_get_graph")
        off = torch.empty(self.n[k] + 1, dtype=torch.int64, device="cuda")
        idx = torch.empty(max(nnz.value, 1), dtype=torch.int32, device="cuda")
        w = torch.empty(max(nnz.value, 1), dtype=torch.float32, device="cuda")
        self._err(lib.leiden_fleet_get_graph(self.ptr, k, _ptr(off), _ptr(idx), _ptr(w), ct.byref(nnz), _stream()),
                  "leiden_fleet_get_graph")
        return off, idx[:nnz.value], w[:nnz.value]

    def get_state(self, k: int):
        n = self.n[k]
        C = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
        K = torch.empty(max(n, 1), dtype=torch.float64, device="cuda")
        S = torch.empty(max(n, 1), dtype=torch.float64, device="cuda")
        m2 = ct.c_double(0.0)
        self._err(load().leiden_fleet_get_state(self.ptr, k, _ptr(C), _ptr(K), _ptr(S), ct.byref(m2), _stream()),
                  "leiden_fleet_get_state")
        return C[:n], K[:n], S[:n], m2.value

    def close(self):
        if self.ptr:
            load().leiden_fleet_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        if getattr(self, "ptr", None) and _lib is not None:
            _lib.leiden_fleet_destroy(self.ptr)
            self.ptr = None
