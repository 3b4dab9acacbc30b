"""Uneven batches (per-query w and k, persistent launch, items merged per
query) against the oracle, bit-exact; HIP-graph replays against eager calls;
the autotuner returns a working shape."""
import numpy as np
import pytest

from conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

U32 = 0xFFFFFFFF


def u32(t):
    return t.cpu().numpy().view(np.uint32)


@pytest.fixture(scope="module")
def env(oracle):
    import torch
    from paper_1209_0410_amd import datagen
    from paper_1209_0410_amd.index import Index
    db = datagen.make_db(100_000)
    db[500:520] = db[7]                       # repeated rows: ties and repeated keys
    q = datagen.make_queries(3000)
    gix = Index(torch.from_numpy(db).cuda())
    return dict(db=db, q=q, gq=torch.from_numpy(q).cuda(), gix=gix, oix=oracle.Index(db))


def check_rows(env, ids, dists, w, k, k_stride):
    ids, dists = u32(ids), u32(dists)
    for kk in np.unique(k):
        m = np.nonzero(k == kk)[0]
        rid, rd = env["oix"].search(env["q"][m], int(kk), w[m])
        assert (ids[m, :kk] == rid).all(), kk
        assert (dists[m, :kk] == rd).all(), kk
        assert (ids[m, kk:] == U32).all() and (dists[m, kk:] == U32).all()


def as_gpu(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, np.uint32).view(np.int32)).cuda()


def test_uneven_log_uniform_w_mixed_k(env):
    """The uneven-batch workload: w log-uniform in [8, 512], k in {1, 10, 100}."""
    from paper_1209_0410_amd import datagen
    w, k = datagen.uneven_w_k(3000)
    ids, d = env["gix"].search_uneven(env["gq"], w_per_query=as_gpu(w), k_per_query=as_gpu(k),
                                      k_stride=100)
    check_rows(env, ids, d, w, k, 100)


@pytest.mark.parametrize("chunk,split", [(64, 4), (256, 32), (8192, 32), (64, 1000)])
def test_uneven_multi_item_queries(env, chunk, split):
    """Large windows cut into many items; the merge drops ids seen twice."""
    from paper_1209_0410_amd import capi
    rng = np.random.default_rng(3)
    n = 600
    w = rng.integers(0, 4000, size=n).astype(np.uint32)
    w[:4] = [0, 1, 50_000, 100_000]
    k = rng.choice([1, 5, 10, 16, 17, 64], size=n).astype(np.uint32)
    cfg = capi.hc_uneven_cfg(chunk, split, 0)
    gq = env["gq"][:n].contiguous()
    ids, d = env["gix"].search_uneven(gq, w_per_query=as_gpu(w), k_per_query=as_gpu(k),
                                      k_stride=64, cfg=cfg)
    sub = dict(env, q=env["q"][:n])
    check_rows(sub, ids, d, w, k, 64)


def test_uneven_batch_over_several_scan_tiles(env):
    """9,000 queries: the item offsets are scanned one block per 4,096 queries
    (three tiles, the last one ragged) and the tile sums are scanned after."""
    import torch
    from paper_1209_0410_amd import datagen
    nq = 9000
    q = datagen.make_queries(nq, seed=21)
    rng = np.random.default_rng(21)
    w = np.exp(rng.uniform(np.log(8), np.log(64), size=nq)).astype(np.uint32)
    w[4095:4098] = [0, 1, 300]                    # around the first tile edge
    k = rng.choice([1, 10, 100], size=nq).astype(np.uint32)
    ids, d = env["gix"].search_uneven(torch.from_numpy(q).cuda(), w_per_query=as_gpu(w),
                                      k_per_query=as_gpu(k), k_stride=100)
    check_rows(dict(env, q=q), ids, d, w, k, 100)


def test_uneven_fixed_w_and_k_matches_plain_search(env):
    gix, gq = env["gix"], env["gq"]
    a_ids, a_d = gix.search(gq, 10, 64)
    b_ids, b_d = gix.search_uneven(gq, w=64, k=10)
    assert (u32(a_ids) == u32(b_ids)).all() and (u32(a_d) == u32(b_d)).all()


def test_uneven_small_k_stride_path(env):
    """k_stride <= 16 compiles out the LDS top-k."""
    from paper_1209_0410_amd import datagen
    w, _ = datagen.uneven_w_k(3000, seed=9)
    k = np.where(np.arange(3000) % 2 == 0, 1, 16).astype(np.uint32)
    ids, d = env["gix"].search_uneven(env["gq"], w_per_query=as_gpu(w), k_per_query=as_gpu(k),
                                      k_stride=16)
    check_rows(env, ids, d, w, k, 16)


def test_graph_replays_match_eager(env):
    """The whole uneven call captured once and replayed, with eager work and
    synchronisation between replays; every replay equals the eager result."""
    import torch
    from paper_1209_0410_amd import datagen
    from paper_1209_0410_amd.tune import Graph
    gix = env["gix"]
    w, k = datagen.uneven_w_k(3000, seed=11)
    gw, gk = as_gpu(w), as_gpu(k)
    gq = env["gq"]
    sc = gix.uneven_scratch(3000, 100)
    out = (torch.empty((3000, 100), dtype=torch.int32, device="cuda"),
           torch.empty((3000, 100), dtype=torch.int32, device="cuda"))
    ref = gix.search_uneven(gq, w_per_query=gw, k_per_query=gk, k_stride=100)
    ref = (ref[0].clone(), ref[1].clone())
    g = Graph(lambda: gix.search_uneven(gq, w_per_query=gw, k_per_query=gk, k_stride=100,
                                        out=out, scratch=sc))
    for rep in range(4):
        out[0].fill_(0)
        out[1].fill_(0)
        gix.search(gq, 10, 32)                 # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out[0], ref[0]) and torch.equal(out[1], ref[1]), rep


def test_graph_of_plain_search(env):
    import torch
    from paper_1209_0410_amd.tune import Graph
    gix, gq = env["gix"], env["gq"]
    sc = gix.scratch(3000)
    out = (torch.empty((3000, 10), dtype=torch.int32, device="cuda"),
           torch.empty((3000, 10), dtype=torch.int32, device="cuda"))
    ref = gix.search(gq, 10, 40)
    ref = (ref[0].clone(), ref[1].clone())
    g = Graph(lambda: gix.search(gq, 10, 40, out=out, scratch=sc))
    for rep in range(3):
        out[0].zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out[0], ref[0]) and torch.equal(out[1], ref[1]), rep


def test_tuner_picks_a_working_shape(env, tmp_path):
    from paper_1209_0410_amd import datagen
    from paper_1209_0410_amd.tune import Tuner
    w, k = datagen.uneven_w_k(3000, seed=13)
    gw, gk = as_gpu(w), as_gpu(k)
    t = Tuner(str(tmp_path / "tune.json"))
    cfg, entry = t.best(env["gix"], env["gq"], gw, gk, sample=1000)
    assert entry["ms"] <= entry["default_ms"]
    ids, d = env["gix"].search_uneven(env["gq"], w_per_query=gw, k_per_query=gk, k_stride=100,
                                      cfg=cfg)
    check_rows(env, ids, d, w, k, 100)
    cfg2, entry2 = Tuner(str(tmp_path / "tune.json")).best(env["gix"], env["gq"], gw, gk)
    assert tuple(entry2["cfg"]) == tuple(entry["cfg"])
