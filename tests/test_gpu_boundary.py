"""GPU tests of the C boundary beyond the method itself: the pure marking
call, the caller's allocator (every device allocation of a handle comes from
it), calls on different streams, and the state a handle is left in when an
update fails after the batch was validated."""
import ctypes as ct

import numpy as np
import pytest
import torch

import oracle
from paper_2405_11658_amd import inputs as gen
from paper_2405_11658_amd import leiden as L

from .gpu_common import dev_batch, ob, og, say, sync_params, to_np

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("mode", ["df", "ds", "nd"])
def test_mark_affected_matches_oracle_and_leaves_handle(mode):
    """Alg. dynamicFrontier / deltaScreening / naiveDynamic flags from the
    pure marking call equal the oracle's, bit for bit, and the handle's graph
    and state are untouched; the update that follows computes the same flags."""
    g = gen.rmat(14, 16, seed=3)
    h = L.leiden_create(g.off, g.idx, g.w, sync_params())
    L.leiden_static(h)
    C0, K0, S0, m20 = L.leiden_get_state(h)
    off0, idx0, w0 = L.leiden_get_graph(h)
    b = gen.random_batch(g, gen.batch_count(g.nnz, 1e-3), seed=11)
    say("mark_affected", mode, "batch", b.size)
    fl = L.leiden_mark_affected(h, dev_batch(b), mode)
    gt, _ = oracle.apply_batch(og(g), ob(b))
    dV, rng, dC = oracle.mark(mode, gt, ob(b), to_np(C0), to_np(K0), to_np(S0), m20)
    assert np.array_equal(to_np(fl["affected"]), dV)
    assert np.array_equal(to_np(fl["in_range"]), rng)
    assert np.array_equal(to_np(fl["changed"]), dC)
    C1, K1, S1, m21 = L.leiden_get_state(h)
    off1, idx1, w1 = L.leiden_get_graph(h)
    assert torch.equal(C0, C1) and torch.equal(K0, K1) and torch.equal(S0, S1) and m20 == m21
    assert torch.equal(off0, off1) and torch.equal(idx0, idx1) and torch.equal(w0, w1)
    _, _, _, tr = L.leiden_update(h, dev_batch(b), mode, trace=True)
    for k in ("affected", "in_range", "changed"):
        assert torch.equal(tr[k], fl[k])


def test_mark_affected_rejects_invalid_batch():
    g = gen.planted_partition(512, 8, 0.2, 0.01, seed=2)
    h = L.leiden_create(g.off, g.idx, g.w, sync_params())
    with pytest.raises(L.LeidenError) as e:
        L.leiden_mark_affected(h, dev_batch(gen.random_batch(g, 4, seed=1)), "df")
    assert e.value.status == L.ESTATE
    L.leiden_static(h)
    u = int(np.repeat(np.arange(g.n), np.diff(g.off))[0])
    v = int(g.idx[0])
    bad = L.make_batch([], [], [u], [v], [1.0])       # inserting an existing edge
    with pytest.raises(L.LeidenError) as e:
        L.leiden_mark_affected(h, bad, "ds")
    assert e.value.status == L.EINVAL


class CountingAllocator:
    """A leiden_allocator over torch's caching allocator that counts what the
    library takes and can refuse one allocation (to force a failure from the
    host, at a chosen point of a call)."""

    def __init__(self, fail_at=None):
        self.base = L.torch_allocator()
        self.count = 0
        self.live = {}
        self.fail_at = fail_at
        self._a = L._ALLOC_FN(self._alloc)
        self._r = L._RELEASE_FN(self._release)
        self.c = L.leiden_allocator(self._a, self._r, None)

    def _alloc(self, ctx, nbytes, stream):
        k = self.count
        self.count += 1
        if self.fail_at is not None and k == self.fail_at:
            return None
        p = self.base._alloc(ctx, nbytes, stream)
        if p:
            self.live[p] = nbytes
        return p

    def _release(self, ctx, ptr, nbytes, stream):
        assert self.live.pop(ptr) == nbytes
        self.base._release(ctx, ptr, nbytes, stream)


def _create(g, params, al):
    lib = L.load()
    off = torch.as_tensor(g.off, device="cuda")
    idx = torch.as_tensor(g.idx, device="cuda")
    w = torch.as_tensor(g.w, device="cuda")
    out = ct.c_void_p()
    st = lib.leiden_create(g.n, g.nnz, L._ptr(off), L._ptr(idx), L._ptr(w), ct.byref(params), ct.byref(al.c),
                           L._stream(), ct.byref(out))
    assert st == L.OK
    return L.Handle(out, g.n)


def test_caller_allocator_provides_every_buffer():
    """All device memory of a handle comes from the caller's allocator and is
    given back at destroy (nothing left outstanding); results are those of the
    oracle (synchronous mode)."""
    g = gen.planted_partition(2048, 32, 0.12, 0.004, seed=5)
    al = CountingAllocator()
    h = _create(g, sync_params(), al)
    C, q, st = L.leiden_static(h)
    ref, _ = oracle.static(og(g), oracle.make_params(sync=True))
    assert np.array_equal(to_np(C), ref.C)
    b = gen.random_batch(g, 20, seed=4)
    C2, q2, _, _ = L.leiden_update(h, dev_batch(b), "df")
    new, _, _, _ = oracle.update(ref, ob(b), "df", oracle.make_params(sync=True))
    assert np.array_equal(to_np(C2), new.C)
    assert al.count > 0 and len(al.live) > 0
    say("allocations", al.count, "outstanding before destroy", len(al.live))
    L.leiden_destroy(h)
    torch.cuda.synchronize()
    assert not al.live


def test_default_allocator_and_streams():
    """A handle on the library's own stream-ordered allocation, used from two
    streams in turn, gives the oracle's results (synchronous mode)."""
    g = gen.rmat(13, 16, seed=7)
    h = L.leiden_create(g.off, g.idx, g.w, sync_params(), allocator=None)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    with torch.cuda.stream(s1):
        C, _, _ = L.leiden_static(h)
    ref, _ = oracle.static(og(g), oracle.make_params(sync=True))
    assert np.array_equal(to_np(C), ref.C)
    state = ref
    cur = g
    for k, s in enumerate((s2, s1, s2)):
        b = gen.random_batch(cur, gen.batch_count(cur.nnz, 1e-3), seed=30 + k)
        with torch.cuda.stream(s):
            C, _, _, _ = L.leiden_update(h, dev_batch(b), "df")
            Cn = to_np(C)
        state, _, _, _ = oracle.update(state, ob(b), "df", oracle.make_params(sync=True))
        assert np.array_equal(Cn, state.C)
        cur = gen.CSR(state.g.n, state.g.off, state.g.idx, state.g.w)
    L.leiden_destroy(h)


def test_failed_update_leaves_graph_without_state():
    """An allocation refused after the batch was validated (forced from the
    host by the allocator) makes the update fail with ENOMEM; the handle then
    holds G^t without a community state: updates return ESTATE until a
    membership is installed, after which they match the oracle again."""
    g = gen.planted_partition(1024, 16, 0.15, 0.005, seed=9)
    b = gen.random_batch(g, 16, seed=2)
    ref0, _ = oracle.static(og(g), oracle.make_params(sync=True))
    # installing a membership allocates only C, K and Sigma, so the update's
    # pass loop allocates its own buffers after the new graph is installed;
    # its last allocation is refused below
    probe = CountingAllocator()
    h = _create(g, sync_params(), probe)
    L.leiden_set_state(h, ref0.C)
    before = probe.count
    L.leiden_update(h, dev_batch(b), "df")
    last = probe.count - 1
    assert last > before
    del h
    al = CountingAllocator(fail_at=last)
    h = _create(g, sync_params(), al)
    L.leiden_set_state(h, ref0.C)
    with pytest.raises(L.LeidenError) as e:
        L.leiden_update(h, dev_batch(b), "df")
    assert e.value.status == L.ENOMEM
    gt, _ = oracle.apply_batch(og(g), ob(b))
    off, idx, w = L.leiden_get_graph(h)
    assert np.array_equal(to_np(off), gt.off) and np.array_equal(to_np(idx), gt.idx)
    b2 = gen.random_batch(gen.CSR(gt.n, gt.off, gt.idx, gt.w), 8, seed=3)
    with pytest.raises(L.LeidenError) as e:
        L.leiden_update(h, dev_batch(b2), "df")
    assert e.value.status == L.ESTATE
    ref, _ = oracle.static(gt, oracle.make_params(sync=True))
    L.leiden_set_state(h, ref.C)
    C, _, _, _ = L.leiden_update(h, dev_batch(b2), "df")
    new, _, _, _ = oracle.update(ref, ob(b2), "df", oracle.make_params(sync=True))
    assert np.array_equal(to_np(C), new.C)
