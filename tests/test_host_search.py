"""The library's host-core search (the CPU side of the cooperative scheduler,
Alg. 3) against the oracle, on the CPU: the lists come from the oracle's
build laid out as the host copy, the handle from hc_index_attach (which
launches nothing).  Bit-exact ids and distances for per-query w and k,
including k beyond the candidates (padding) and w = 0."""
import ctypes as ct

import numpy as np
import pytest

from paper_1209_0410_amd import capi


def aligned(nbytes, align=256):
    raw = np.zeros(nbytes + align, np.uint8)
    off = (-raw.ctypes.data) % align
    return raw[off:off + nbytes]


@pytest.fixture(scope="module")
def setup(oracle):
    from paper_1209_0410_amd import datagen
    db = datagen.make_rows(20_000, 31)
    db[500:510] = db[7]                     # equal keys and distance ties
    q = datagen.make_rows(120, 32)
    q[0] = db[7]
    oix = oracle.Index(db)
    lib = capi.load()
    p, keep = capi.make_params()
    ib = ct.c_size_t()
    assert lib.hc_index_bytes(ct.byref(p), len(db), ct.byref(ib), None) == 0
    buf = aligned(ib.value)
    dbh = np.ascontiguousarray(db)
    h = ct.c_void_p()
    assert lib.hc_index_attach(ct.byref(p), dbh.ctypes.data_as(ct.c_void_p), len(db),
                               buf.ctypes.data_as(ct.c_void_p), ib.value, ct.byref(h)) == 0
    sz = ct.c_size_t()
    assert lib.hc_host_index_bytes(h, ct.byref(sz)) == 0
    n = len(db)
    assert sz.value == 8 * n * 20
    lists = np.zeros(sz.value, np.uint8)
    keys = lists[:16 * 8 * n].view(np.uint64).reshape(8, n, 2)
    keys[:, :, 0] = oix.hi
    keys[:, :, 1] = oix.lo
    lists[16 * 8 * n:].view(np.uint32).reshape(8, n)[:] = oix.ids
    yield dict(db=dbh, q=q, oix=oix, lib=lib, h=h, lists=lists, keep=(buf, keep))
    lib.hc_index_destroy(h)


def host_search(S, q, w, k, k_stride):
    nq = len(q)
    ids = np.zeros((nq, k_stride), np.uint32)
    d = np.zeros((nq, k_stride), np.uint32)
    wv = np.ascontiguousarray(w, np.uint32)
    kv = np.ascontiguousarray(k, np.uint32)
    qq = np.ascontiguousarray(q)
    vp = ct.c_void_p
    st = S["lib"].hc_host_search(S["h"], S["lists"].ctypes.data_as(vp),
                                 S["db"].ctypes.data_as(vp), qq.ctypes.data_as(vp), nq, 0,
                                 wv.ctypes.data_as(vp), 0, kv.ctypes.data_as(vp), k_stride,
                                 ids.ctypes.data_as(vp), d.ctypes.data_as(vp))
    assert st == 0
    return ids, d


def test_host_search_bit_exact(setup):
    S = setup
    rng = np.random.default_rng(4)
    nq = len(S["q"])
    w = rng.integers(0, 300, size=nq).astype(np.uint32)
    w[:3] = [0, 1, 20_000]
    k = rng.choice([1, 10, 100], size=nq).astype(np.uint32)
    ids, d = host_search(S, S["q"], w, k, 100)
    for kk in (1, 10, 100):
        m = np.nonzero(k == kk)[0]
        for wv in np.unique(w[m]):
            mm = m[w[m] == wv]
            rid, rd = S["oix"].search(S["q"][mm], int(kk), int(wv))
            assert (ids[mm, :kk] == rid).all() and (d[mm, :kk] == rd).all(), (kk, wv)
    # padding beyond k
    for i in range(nq):
        assert (ids[i, k[i]:] == 0xFFFFFFFF).all() and (d[i, k[i]:] == 0xFFFFFFFF).all()


def test_host_search_rejects_bad_arguments(setup):
    S = setup
    lib, vp = S["lib"], ct.c_void_p
    out = np.zeros((1, 10), np.uint32)
    q = np.ascontiguousarray(S["q"][:1])
    args = [S["h"], S["lists"].ctypes.data_as(vp), S["db"].ctypes.data_as(vp),
            q.ctypes.data_as(vp), 1, 16, None, 10, None, 10, out.ctypes.data_as(vp),
            out.ctypes.data_as(vp)]
    assert lib.hc_host_search(*args) == 0
    bad = list(args)
    bad[9] = 0                                        # k_stride 0
    assert lib.hc_host_search(*bad) == capi.HC_ERR_INVALID
    bad = list(args)
    bad[7] = 11                                       # k_fixed > k_stride
    assert lib.hc_host_search(*bad) == capi.HC_ERR_INVALID
    bad = list(args)
    bad[1] = None
    assert lib.hc_host_search(*bad) == capi.HC_ERR_INVALID
