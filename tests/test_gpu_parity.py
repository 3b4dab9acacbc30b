"""GPU parity: every step of the HIP search path, called through the C ABI,
against the CPU oracle on the same seeded inputs.  Integer work, so the bar
is bit-exact: keys, sorted lists, positions, candidate sets, distances,
top-k ids and distances (ties by id)."""
import numpy as np
import pytest

from conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

U32 = 0xFFFFFFFF


def u32(t):
    return t.cpu().numpy().view(np.uint32)


def u64(t):
    return t.cpu().numpy().view(np.uint64)


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    return torch


@pytest.fixture(scope="module")
def c1(oracle, torch_mod):
    """Plain method, tiny: N = 100,000, Q = 1,000 (mixture seeds 1 and 2)."""
    from paper_1209_0410_amd import datagen
    from paper_1209_0410_amd.index import Index
    db = datagen.make_db(100_000)
    q = datagen.make_queries(1000)
    dev = torch_mod.device("cuda:0")
    gdb = torch_mod.from_numpy(db).to(dev)
    gq = torch_mod.from_numpy(q).to(dev)
    print(f"[c1] building GPU index n={db.shape[0]}", flush=True)
    gix = Index(gdb)
    oix = oracle.Index(db)
    return dict(db=db, q=q, gdb=gdb, gq=gq, gix=gix, oix=oix)


def test_encode_keys_bit_exact(c1, oracle, torch_mod):
    from paper_1209_0410_amd.index import encode_keys
    keys = u64(encode_keys(c1["gdb"]))                   # (n, 8, 2) {hi, lo}
    hi, lo = oracle.keys(c1["db"], oracle.Params())
    assert (keys[:, :, 0] == hi).all() and (keys[:, :, 1] == lo).all()


def test_encode_keys_random_points(oracle, torch_mod):
    """Uniform random bytes (all 256 values per coordinate) and extremes."""
    from paper_1209_0410_amd.index import encode_keys
    rng = np.random.default_rng(7)
    rows = rng.integers(0, 256, size=(50_000, 128), dtype=np.uint8)
    rows[0] = 0
    rows[1] = 255
    rows[2] = np.arange(128) % 256
    g = u64(encode_keys(torch_mod.from_numpy(rows).cuda()))
    hi, lo = oracle.keys(rows, oracle.Params())
    assert (g[:, :, 0] == hi).all() and (g[:, :, 1] == lo).all()


def test_sorted_lists_bit_exact(c1):
    gix, oix = c1["gix"], c1["oix"]
    for c in range(8):
        keys, ids = gix.curve(c)
        k = u64(keys)
        assert (k[:, 0] == oix.hi[c]).all() and (k[:, 1] == oix.lo[c]).all(), c
        assert (u32(ids) == oix.ids[c]).all(), c


def test_positions_bit_exact(c1):
    pos = u32(c1["gix"].positions(c1["gq"]))
    assert (pos == c1["oix"].positions(c1["q"])).all()


@pytest.mark.parametrize("w", [1, 16, 64, 256])
def test_candidate_sets_bit_exact(c1, w):
    counts, ids = c1["gix"].candidates(c1["gq"][:300], w)
    counts = u32(counts)
    ids = u32(ids)
    ref = c1["oix"].candidates(c1["q"][:300], w)
    for i, r in enumerate(ref):
        assert counts[i] == len(r)
        assert (np.sort(ids[i, :counts[i]]) == r).all()


def test_candidate_limits(c1, torch_mod):
    """The export's limits as the header states them: stride above 4096 is
    refused; with a w per query, a query whose window slots exceed the stride
    is flagged 0xFFFFFFFF and the others are exact."""
    from paper_1209_0410_amd import capi
    with pytest.raises(capi.HcError) as e:
        c1["gix"].candidates(c1["gq"][:4], 300, stride=4097)
    assert e.value.status == capi.HC_ERR_UNSUPPORTED
    with pytest.raises(capi.HcError) as e:
        c1["gix"].candidates(c1["gq"][:4], 300, stride=4000)
    assert e.value.status == capi.HC_ERR_SIZE
    w = np.array([16, 300, 256, 1], np.uint32)        # 16 * 300 > 4096 slots
    gw = torch_mod.from_numpy(w.view(np.int32)).cuda()
    counts, ids = c1["gix"].candidates(c1["gq"][:4], 0, w_per_query=gw, stride=4096)
    counts, ids = u32(counts), u32(ids)
    assert counts[1] == U32
    for i in (0, 2, 3):
        ref = c1["oix"].candidates(c1["q"][i:i + 1], int(w[i]))[0]
        assert counts[i] == len(ref) and (np.sort(ids[i, :counts[i]]) == ref).all()


@pytest.mark.parametrize("k,w", [(10, 64), (1, 16), (10, 1), (16, 256), (17, 64),
                                 (100, 64), (256, 40), (10, 300), (10, 600), (5, 2000)])
def test_search_bit_exact(c1, k, w):
    nq = 1000 if w <= 300 else 200
    ids, d = c1["gix"].search(c1["gq"][:nq], k, w)
    rid, rd = c1["oix"].search(c1["q"][:nq], k, w)
    assert (u32(ids) == rid).all()
    assert (u32(d) == rd).all()


def test_per_query_w_bit_exact(c1, torch_mod):
    rng = np.random.default_rng(3)
    w = rng.integers(0, 400, size=1000).astype(np.uint32)
    w[:5] = [0, 1, 2, 700, 5000]
    gw = torch_mod.from_numpy(w.view(np.int32)).cuda()
    for hint in [0, 32, 256]:
        ids, d = c1["gix"].search(c1["gq"], 10, hint, w_per_query=gw)
        rid, rd = c1["oix"].search(c1["q"], 10, w)
        assert (u32(ids) == rid).all() and (u32(d) == rd).all(), hint


def test_brute_force_bit_exact(c1, oracle):
    from paper_1209_0410_amd.index import brute_force
    ids, d = brute_force(c1["gdb"], c1["gq"][:200], 10)
    rid, rd = oracle.brute_force(c1["db"], c1["q"][:200], 10)
    assert (u32(ids) == rid).all() and (u32(d) == rd).all()


def test_deterministic_and_batch_independent(c1):
    gix, gq = c1["gix"], c1["gq"]
    a_ids, a_d = gix.search(gq, 10, 64)
    b_ids, b_d = gix.search(gq, 10, 64)
    assert (u32(a_ids) == u32(b_ids)).all() and (u32(a_d) == u32(b_d)).all()
    alone_ids, alone_d = gix.search(gq[17:18].contiguous(), 10, 64)
    assert (u32(alone_ids)[0] == u32(a_ids)[17]).all()


@pytest.mark.parametrize("n", [1, 7, 64, 65, 521, 1000, 4097, 65537])
def test_small_shapes_bit_exact(oracle, torch_mod, n):
    from paper_1209_0410_amd import datagen
    from paper_1209_0410_amd.index import Index
    db = datagen.make_rows(n, 11)
    if n > 100:
        db[50::50] = db[3]                     # forced duplicate keys and distance ties
    q = datagen.make_rows(300, 12)
    q[0] = 0
    q[1] = 255
    q[2] = db[min(3, n - 1)]
    print(f"[small] n={n}", flush=True)
    gix = Index(torch_mod.from_numpy(db).cuda())
    oix = oracle.Index(db)
    for c in range(8):
        keys, ids = gix.curve(c)
        assert (u32(ids) == oix.ids[c]).all()
    gq = torch_mod.from_numpy(q).cuda()
    assert (u32(gix.positions(gq)) == oix.positions(q)).all()
    for k, w in [(10, 1), (10, 8), (20, 64), (3, n)]:
        ids, d = gix.search(gq, k, w)
        rid, rd = oix.search(q, k, w)
        assert (u32(ids) == rid).all() and (u32(d) == rd).all(), (k, w)


def test_full_window_is_exact_knn(oracle, torch_mod):
    from paper_1209_0410_amd import datagen
    from paper_1209_0410_amd.index import Index
    db = datagen.make_rows(3000, 21)
    db[100:110] = db[7]
    q = datagen.make_rows(100, 22)
    gix = Index(torch_mod.from_numpy(db).cuda())
    ids, d = gix.search(torch_mod.from_numpy(q).cuda(), 10, 3000)
    rid, rd = oracle.brute_force(db, q, 10)
    assert (u32(ids) == rid).all() and (u32(d) == rd).all()


@pytest.mark.parametrize("k,w", [(10, 64), (1, 16), (10, 1), (16, 256), (4, 3000), (10, 0),
                                 (7, 20_000)])
def test_banded_path_bit_exact(c1, k, w):
    """The banded execution (queries grouped by place in each list) gives the
    gather search's results exactly."""
    ids, d = c1["gix"].search(c1["gq"], k, w, path=2)
    rid, rd = c1["oix"].search(c1["q"], k, w)
    assert (u32(ids) == rid).all()
    assert (u32(d) == rd).all()


def test_banded_path_per_query_w(c1, torch_mod):
    rng = np.random.default_rng(17)
    w = rng.integers(0, 3000, size=1000).astype(np.uint32)
    w[:3] = [0, 1, 90_000]
    gw = torch_mod.from_numpy(w.view(np.int32)).cuda()
    ids, d = c1["gix"].search(c1["gq"], 10, 512, w_per_query=gw, path=2)
    rid, rd = c1["oix"].search(c1["q"], 10, w)
    assert (u32(ids) == rid).all() and (u32(d) == rd).all()


def test_auto_path_matches_both(c1):
    for w in (8, 600):
        a = c1["gix"].search(c1["gq"], 10, w, path=0)
        g = c1["gix"].search(c1["gq"], 10, w, path=1)
        b = c1["gix"].search(c1["gq"], 10, w, path=2)
        for x, y in ((a, g), (g, b)):
            assert (u32(x[0]) == u32(y[0])).all() and (u32(x[1]) == u32(y[1])).all()


@pytest.mark.parametrize("path", [1, 2])
def test_kernel_events_time_the_main_kernel_only(c1, torch_mod, path):
    """Events recorded by the library around the search's main kernel: the
    results do not change, the kernel's time lies inside the call's, and only
    one event set is rejected."""
    import ctypes as ct
    from paper_1209_0410_amd import capi
    torch = torch_mod
    gix, gq = c1["gix"], c1["gq"]
    ref = gix.search(gq, 10, 300, path=path)
    sc = gix.scratch(gq.shape[0])
    out = (torch.empty_like(ref[0]), torch.empty_like(ref[1]))
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    st = torch.cuda.current_stream()
    for e in ev:
        e.record(st)
    gix.encode_queries(gq, sc)
    ev[0].record(st)
    gix.set_kernel_events(ev[1], ev[2])
    gix.search_encoded(gq, 10, 300, out, sc, path=path)
    gix.set_kernel_events()
    ev[3].record(st)
    torch.cuda.synchronize()
    call, kern = ev[0].elapsed_time(ev[3]), ev[1].elapsed_time(ev[2])
    assert 0 < kern <= call
    assert (u32(out[0]) == u32(ref[0])).all() and (u32(out[1]) == u32(ref[1])).all()
    assert capi.load().hc_index_set_kernel_events(gix.handle, ct.c_void_p(ev[1].cuda_event),
                                                 None) == capi.HC_ERR_INVALID
    again = gix.search(gq, 10, 300, path=path)
    assert (u32(again[0]) == u32(ref[0])).all()


@pytest.mark.parametrize("k,w", [(10, 64), (1, 16), (16, 256), (4, 3000), (10, 0), (7, 20_000)])
def test_rowstore_banded_bit_exact(c1, k, w):
    """With the row store attached (rows in list order, read contiguously), the
    banded search gives the same results."""
    gix = c1["gix"]
    gix.attach_rowstore()
    try:
        ids, d = gix.search(c1["gq"], k, w, path=2)
    finally:
        gix.detach_rowstore()
    rid, rd = c1["oix"].search(c1["q"], k, w)
    assert (u32(ids) == rid).all() and (u32(d) == rd).all()


@pytest.mark.parametrize("k", [1, 10, 100])
def test_small_batch_long_windows_as_work_items(c1, torch_mod, k):
    """A batch too small to keep the device busy with one wavefront per query,
    at long windows (2 w x 8 curves >= 32,768 slots per query), runs as work
    items on the automatic path.  Its results equal the gather kernel's
    (forced path) on every query, with a fixed w and with a w per query, and
    the oracle's at k = 10."""
    gix = c1["gix"]
    gq = c1["gq"][:200].contiguous()
    print(f"[items] k={k}", flush=True)
    ids, d = gix.search(gq, k, 3000)
    gids, gd = gix.search(gq, k, 3000, path=1)
    assert (u32(ids) == u32(gids)).all() and (u32(d) == u32(gd)).all()
    g = torch_mod.Generator().manual_seed(29)
    wq = torch_mod.randint(2100, 6000, (200,), generator=g, dtype=torch_mod.int32).cuda()
    ids, d = gix.search(gq, k, 3000, w_per_query=wq)
    gids, gd = gix.search(gq, k, 3000, w_per_query=wq, path=1)
    assert (u32(ids) == u32(gids)).all() and (u32(d) == u32(gd)).all()
    if k == 10:
        rid, rd = c1["oix"].search(c1["q"][:200], k, 3000)
        ids, d = gix.search(gq, k, 3000)
        assert (u32(ids) == rid).all() and (u32(d) == rd).all()


def test_rowstore_banded_last_round_split(c1, torch_mod):
    """A batch whose banded grid ends with a short round: the last groups'
    unions are dealt out over several blocks and their lists merged after the
    main kernel.  With 256-query groups (w >= 8192) 18,176 queries make
    71 x 8 = 568 groups, 56 past the 512 (k <= 10) or 256 (k = 16) blocks
    resident at once on MI355X.  Every query's results equal the gather
    kernel's, and the oracle's on a sample."""
    from paper_1209_0410_amd import datagen
    q = datagen.make_queries(18_176, seed=23)
    gq = torch_mod.from_numpy(q).cuda()
    gix = c1["gix"]
    gix.attach_rowstore()
    try:
        for k in (1, 10, 16):
            print(f"[last round] k={k}", flush=True)
            ids, d = gix.search(gq, k, 9000, path=2)
            gids, gd = gix.search(gq, k, 9000, path=1)
            assert (u32(ids) == u32(gids)).all() and (u32(d) == u32(gd)).all(), k
            if k == 10:
                sample = np.arange(0, q.shape[0], 61)
                rid, rd = c1["oix"].search(q[sample], k, 9000)
                assert (u32(ids)[sample] == rid).all() and (u32(d)[sample] == rd).all()
    finally:
        gix.detach_rowstore()


@pytest.mark.parametrize("n", [1, 65, 4097])
def test_rowstore_small_shapes_and_per_query_w(oracle, torch_mod, n):
    from paper_1209_0410_amd import datagen
    from paper_1209_0410_amd.index import Index
    db = datagen.make_rows(n, 41)
    if n > 100:
        db[50::50] = db[3]
    q = datagen.make_rows(300, 42)
    q[0] = db[0]
    print(f"[rowstore] n={n}", flush=True)
    gix = Index(torch_mod.from_numpy(db).cuda())
    gix.attach_rowstore()
    oix = oracle.Index(db)
    gq = torch_mod.from_numpy(q).cuda()
    w = np.random.default_rng(43).integers(0, 2 * n + 2, size=300).astype(np.uint32)
    gw = torch_mod.from_numpy(w.view(np.int32)).cuda()
    ids, d = gix.search(gq, 10, int(w.max()), w_per_query=gw, path=2)
    rid, rd = oix.search(q, 10, w)
    assert (u32(ids) == rid).all() and (u32(d) == rd).all()
