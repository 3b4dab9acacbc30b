"""GPU parity of the Z-order comparison curve and of incremental insertion.

- Z-order (Sec. 2.2.1, the coordinates' bits intercalated): keys, sorted
  lists and search results bit-exact against the oracle's Z-order index.
- Insertion (Alg. 1 run incrementally, Sec. 3.1 / Sec. 4.1): an index over the
  first n rows plus rows n .. n + m - 1 inserted gives the lists a full build
  over n + m rows gives, bit for bit (oracle and GPU build), including equal
  keys across the old and the new rows, twice in a row, and on the Z-order
  curve; searches on the result match the oracle.
"""
import ctypes as ct

import numpy as np
import pytest

from conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def u32(t):
    return t.cpu().numpy().view(np.uint32)


def u64(t):
    return t.cpu().numpy().view(np.uint64)


@pytest.fixture(scope="module")
def data():
    from paper_1209_0410_amd import datagen
    db = datagen.make_db(100_000)
    q = datagen.make_queries(500)
    return db, q


def same_lists(gix, oix):
    for c in range(8):
        keys, ids = gix.curve(c)
        k = u64(keys)
        assert (k[:, 0] == oix.hi[c]).all() and (k[:, 1] == oix.lo[c]).all(), c
        assert (u32(ids) == oix.ids[c]).all(), c


def test_zorder_keys_bit_exact(oracle, data):
    import torch
    from paper_1209_0410_amd.index import encode_keys
    db, _ = data
    rows = np.concatenate([db[:20_000], np.random.default_rng(3).integers(
        0, 256, size=(5_000, 128), dtype=np.uint8)])
    rows[-1] = 255
    rows[-2] = 0
    g = u64(encode_keys(torch.from_numpy(rows).cuda(), curve="zorder"))
    hi, lo = oracle.keys(rows, oracle.Params(curve="zorder"))
    assert (g[:, :, 0] == hi).all() and (g[:, :, 1] == lo).all()


def test_zorder_index_and_search_bit_exact(oracle, data):
    import torch
    from paper_1209_0410_amd.index import Index
    db, q = data
    gix = Index(torch.from_numpy(db).cuda(), curve="zorder")
    oix = oracle.Index(db, oracle.Params(curve="zorder"))
    same_lists(gix, oix)
    gq = torch.from_numpy(q).cuda()
    for k, w, path in [(10, 64, 1), (1, 16, 1), (100, 40, 1), (10, 600, 2), (10, 600, 1)]:
        ids, d = gix.search(gq, k, w, path=path)
        rid, rd = oix.search(q, k, w)
        assert (u32(ids) == rid).all() and (u32(d) == rd).all(), (k, w, path)


@pytest.mark.parametrize("n0,m", [(99_999, 1), (96_000, 4_000), (50_000, 50_000),
                                  (1, 4_097), (64, 1)])
def test_insert_equals_full_build(oracle, data, n0, m):
    import torch
    from paper_1209_0410_amd.index import Index
    db, _ = data
    rows = db[:n0 + m].copy() if n0 + m <= len(db) else None
    if rows is None:
        pytest.skip("sizes")
    if m > 10:
        rows[n0::97] = rows[: len(rows[n0::97])]      # new rows equal to old rows: equal keys
    print(f"[insert] n0={n0} m={m}", flush=True)
    g = torch.from_numpy(rows).cuda()
    base = Index(g[:n0])
    ins = base.insert(g)
    full = Index(g)
    oix = oracle.Index(rows)
    same_lists(ins, oix)
    for c in range(8):
        a_keys, a_ids = ins.curve(c)
        b_keys, b_ids = full.curve(c)
        assert torch.equal(a_keys, b_keys) and torch.equal(a_ids, b_ids)
    # the old index is untouched and still searchable
    same_lists(base, oracle.Index(rows[:n0]))


def test_insert_twice_then_search(oracle, data):
    import torch
    from paper_1209_0410_amd.index import Index
    db, q = data
    g = torch.from_numpy(db).cuda()
    ix = Index(g[:60_000]).insert(g[:80_000]).insert(g)
    oix = oracle.Index(db)
    same_lists(ix, oix)
    gq = torch.from_numpy(q).cuda()
    for k, w in [(10, 64), (10, 700)]:
        ids, d = ix.search(gq, k, w)
        rid, rd = oix.search(q, k, w)
        assert (u32(ids) == rid).all() and (u32(d) == rd).all(), (k, w)


def test_zorder_rowstore_and_inserted_rowstore(oracle, data):
    """The row store (tiles copied into LDS) on a Z-order index and on an index
    made by insertion: banded searches stay bit-exact."""
    import torch
    from paper_1209_0410_amd.index import Index
    db, q = data
    gq = torch.from_numpy(q).cuda()
    g = torch.from_numpy(db).cuda()
    zix = Index(g, curve="zorder")
    zix.attach_rowstore()
    zo = oracle.Index(db, oracle.Params(curve="zorder"))
    for k, w in [(10, 600), (4, 9000)]:
        ids, d = zix.search(gq, k, w, path=2)
        rid, rd = zo.search(q, k, w)
        assert (u32(ids) == rid).all() and (u32(d) == rd).all(), ("zorder", k, w)
    ins = Index(g[:70_000]).insert(g)
    ins.attach_rowstore()
    ho = oracle.Index(db)
    for k, w in [(10, 600), (16, 9000)]:
        ids, d = ins.search(gq, k, w, path=2)
        rid, rd = ho.search(q, k, w)
        assert (u32(ids) == rid).all() and (u32(d) == rd).all(), ("inserted", k, w)


def test_insert_zorder(oracle, data):
    import torch
    from paper_1209_0410_amd.index import Index
    db, _ = data
    g = torch.from_numpy(db[:30_000]).cuda()
    ix = Index(g[:25_000], curve="zorder").insert(g)
    same_lists(ix, oracle.Index(db[:30_000], oracle.Params(curve="zorder")))


def test_insert_rejects_overlap_and_bad_sizes(data):
    import torch
    from paper_1209_0410_amd import capi
    from paper_1209_0410_amd.index import Index
    db, _ = data
    g = torch.from_numpy(db[:2_000]).cuda()
    ix = Index(g[:1_000])
    lib = capi.load()
    ib, sb = ct.c_size_t(), ct.c_size_t()
    assert lib.hc_insert_bytes(ix.handle, 1_000, ct.byref(ib), ct.byref(sb)) == 0
    assert lib.hc_insert_bytes(ix.handle, 0, ct.byref(ib), ct.byref(sb)) == capi.HC_ERR_INVALID
    scratch = torch.empty(sb.value + 256, dtype=torch.uint8, device="cuda")
    off = (-scratch.data_ptr()) % 256
    sp = ct.c_void_p(scratch.data_ptr() + off)
    h = ct.c_void_p()
    # the new index may not be written over the old one
    st = lib.hc_insert_rows(ix.handle, ct.c_void_p(g.data_ptr()), 1_000,
                            ct.c_void_p(ix.buf.data_ptr()), ib.value, sp, sb.value, None,
                            ct.byref(h))
    assert st == capi.HC_ERR_INVALID
    buf = torch.empty(ib.value + 256, dtype=torch.uint8, device="cuda")
    bp = ct.c_void_p(buf.data_ptr() + (-buf.data_ptr()) % 256)
    assert lib.hc_insert_rows(ix.handle, ct.c_void_p(g.data_ptr()), 1_000, bp, ib.value - 1,
                              sp, sb.value, None, ct.byref(h)) == capi.HC_ERR_SIZE
    assert lib.hc_insert_rows(ix.handle, ct.c_void_p(g.data_ptr()), 1_000, bp, ib.value,
                              sp, sb.value - 1, None, ct.byref(h)) == capi.HC_ERR_SIZE
