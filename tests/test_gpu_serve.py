"""The continuous-batching request loop: every request's result is the same
as when it is searched alone (integer results, bit-exact), under a
fluctuating arrival rate, with and without a tight HBM budget, with a learned
w per request."""
import numpy as np
import pytest

from conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def u32(t):
    return t.cpu().numpy().view(np.uint32)


@pytest.fixture(scope="module")
def env(oracle):
    import torch
    from paper_1209_0410_amd import datagen
    from paper_1209_0410_amd.index import Index
    db = datagen.make_db(50_000)
    gix = Index(torch.from_numpy(db).cuda())
    R = 4000
    q = datagen.make_queries(R, seed=21)
    ks = np.random.default_rng(22).choice([1, 10, 100], size=R).astype(np.uint32)
    return dict(db=db, gix=gix, q=q, ks=ks, oix=oracle.Index(db))


def alone(gix, q, ks, w, k_stride=100):
    """Each request searched by itself."""
    import torch
    ids = np.zeros((len(q), k_stride), np.uint32)
    d = np.zeros((len(q), k_stride), np.uint32)
    for i in range(len(q)):
        gi, gd = gix.search_uneven(torch.from_numpy(q[i:i + 1]).cuda(), w=int(w[i]),
                                   k=int(ks[i]), k_stride=k_stride)
        ids[i], d[i] = u32(gi)[0], u32(gd)[0]
    return ids, d


def test_results_equal_alone_and_in_the_mix(env):
    from paper_1209_0410_amd.serve import Server, sinusoidal_arrivals
    arr = sinusoidal_arrivals(0.4, 2000, 20000, 0.4, seed=23)
    R = min(len(arr), len(env["q"]))
    arr = arr[:R]
    srv = Server(env["gix"], w_fixed=24, k_stride=100, max_batch=512, slots=3)
    stats, (ids, d) = srv.run(arr, env["q"][:R], env["ks"][:R])
    assert stats["requests"] == R and stats["batches"] > 1
    w = np.full(R, 24)
    sel = np.arange(0, R, 7)
    ai, ad = alone(env["gix"], env["q"][sel], env["ks"][sel], w[sel])
    assert (ids[sel] == ai).all() and (d[sel] == ad).all()
    # and against the oracle, per k
    for kk in (1, 10, 100):
        m = sel[env["ks"][sel] == kk]
        rid, rd = env["oix"].search(env["q"][m], int(kk), 24)
        assert (ids[m, :kk] == rid).all() and (d[m, :kk] == rd).all()
    assert np.isfinite(stats["p99_ms"]) and stats["p99_ms"] >= stats["p50_ms"]


def test_tight_hbm_budget_limits_batches(env):
    from paper_1209_0410_amd.serve import HbmBudget, Server
    R = 1500
    arr = np.zeros(R)                       # everything arrives at once
    srv2 = Server(env["gix"], w_fixed=16, k_stride=100, max_batch=1024, slots=1)
    budget = HbmBudget(srv2.batch_bytes(200))
    srv = Server(env["gix"], w_fixed=16, k_stride=100, max_batch=1024, slots=3, budget=budget)
    assert budget.buf.numel() == budget.budget == srv.batch_bytes(200)
    stats, (ids, d) = srv.run(arr, env["q"][:R], env["ks"][:R])
    assert stats["max_batch"] == 200 and budget.peak <= budget.budget
    assert budget.used == 0 and budget.largest() == budget.budget
    assert stats["admission_waits"] > 0
    _, (ids2, d2) = srv2.run(arr, env["q"][:R], env["ks"][:R])
    assert (ids == ids2).all() and (d == d2).all()


def test_budget_below_one_request_is_an_error(env):
    from paper_1209_0410_amd.serve import HbmBudget, Server
    srv = Server(env["gix"], w_fixed=16, k_stride=100, max_batch=64, slots=1,
                 budget=HbmBudget(1000))
    with pytest.raises(RuntimeError):
        srv.run(np.zeros(10), env["q"][:10], env["ks"][:10])


def test_learned_w_per_request_in_the_mix(env):
    import torch
    from paper_1209_0410_amd import learned
    from paper_1209_0410_amd.serve import Server, sinusoidal_arrivals
    model = learned.WModel(torch.device("cuda:0"), seed=5, w_min=8, w_max=256)
    feats = learned.features(env["gix"], torch.from_numpy(env["q"]).cuda(), 10)
    model.set_norm(feats)
    model.delta = 5.0
    arr = sinusoidal_arrivals(0.3, 2000, 15000, 0.3, seed=24)
    R = min(len(arr), 1500)
    srv = Server(env["gix"], model=model, w_fixed=32, k_stride=100, max_batch=256, slots=2)
    stats, (ids, d) = srv.run(arr[:R], env["q"][:R], env["ks"][:R])
    # the w each request got depends on its own features only (with k capped
    # at the depth the model is trained for)
    gq = torch.from_numpy(env["q"][:R]).cuda()
    gk = torch.from_numpy(np.minimum(env["ks"][:R], 10).astype(np.uint32).view(np.int32)).cuda()
    f = learned.features(env["gix"], gq, 0, gk)
    w = u32(model.windows(f, w_fallback=32))
    sel = np.arange(0, R, 9)
    ai, ad = alone(env["gix"], env["q"][sel], env["ks"][sel], w[sel])
    assert (ids[sel] == ai).all() and (d[sel] == ad).all()


def test_host_search_equals_gpu(env):
    """The host-core search (the CPU side of the cooperative scheduler) gives the
    GPU's rows bit for bit, from a host copy of the device lists."""
    import torch
    from paper_1209_0410_amd.index import HostSearch
    host = HostSearch(env["gix"], env["db"])
    rng = np.random.default_rng(31)
    R = 600
    q = env["q"][:R]
    w = rng.integers(0, 200, size=R).astype(np.uint32)
    w[:2] = [0, 60_000]
    ks = env["ks"][:R]
    gi, gd = env["gix"].search_uneven(
        torch.from_numpy(q).cuda(), w_per_query=torch.from_numpy(w.view(np.int32)).cuda(),
        k_per_query=torch.from_numpy(ks.view(np.int32)).cuda(), k_stride=100)
    hi_, hd = host.search(q, k_stride=100, w_per_query=w, k_per_query=ks)
    assert (u32(gi) == hi_).all() and (u32(gd) == hd).all()


def test_cooperative_scheduler_same_results(env):
    """A short queue goes to host cores, a burst to the GPU (and to idle host
    cores from the front); every request's row equals its GPU row alone."""
    from paper_1209_0410_amd.index import HostSearch
    from paper_1209_0410_amd.serve import Server
    host = HostSearch(env["gix"], env["db"])
    R = 2400
    arr = np.concatenate([np.arange(400) * 1e-3, np.full(R - 400, 0.45)])
    srv = Server(env["gix"], w_fixed=24, k_stride=100, max_batch=512, slots=2, host=host,
                 cpu_workers=4)
    stats, (ids, d) = srv.run(arr, env["q"][:R], env["ks"][:R])
    assert stats["requests"] == R
    assert stats["on_host_cores"] > 0 and stats["batches"] > 0
    w = np.full(R, 24)
    sel = np.arange(0, R, 5)
    ai, ad = alone(env["gix"], env["q"][sel], env["ks"][sel], w[sel])
    assert (ids[sel] == ai).all() and (d[sel] == ad).all()


def test_batch_route_banded_equals_alone(oracle):
    """The batch route at a wide window: one batch of 30,000 requests packed
    by k, each k class a banded search over the row store (k = 100 in two
    passes), then smaller batches arriving over time (classes of at least 512
    banded, smaller ones gathered); every row equals the uneven route's (the
    gather kernel), the sample the oracle's."""
    import torch
    from paper_1209_0410_amd import datagen
    from paper_1209_0410_amd.index import Index
    from paper_1209_0410_amd.serve import Server, sinusoidal_arrivals
    n, R, w = 200_000, 30_000, 3_000
    db = datagen.make_db(n)
    gix = Index(torch.from_numpy(db).cuda())
    gix.attach_rowstore()
    q = datagen.make_queries(R, seed=25)
    ks = np.random.default_rng(26).choice([1, 10, 100], size=R).astype(np.uint32)
    # each k class of the whole batch is large enough to band
    for kk in (1, 10, 100):
        m = int((ks == kk).sum())
        sc = gix.new_scratch(m, 100)
        assert gix.path(m, int(kk), w, sc.numel()) == 2
        del sc
    srv = Server(gix, w_fixed=w, k_stride=100, max_batch=R, slots=1, route="batch")
    stats, (ids, d) = srv.run(np.zeros(R), q, ks, realtime=False)
    assert stats["batches"] == 1
    ref = Server(gix, w_fixed=w, k_stride=100, max_batch=4096, slots=2)
    _, (rids, rd) = ref.run(np.zeros(R), q, ks, realtime=False)
    assert (ids == rids).all() and (d == rd).all()
    sel = np.arange(0, R, 211)
    oix = oracle.Index(db)
    for kk in (1, 10, 100):
        m = sel[ks[sel] == kk]
        oi, od = oix.search(q[m], int(kk), w)
        assert (ids[m, :kk] == oi).all() and (d[m, :kk] == od).all()
    # arrivals over time with a minimum batch: several batches, same rows
    arr = sinusoidal_arrivals(0.5, 20_000, 80_000, 0.5, seed=27)
    Rt = min(len(arr), 12_000)
    srv2 = Server(gix, w_fixed=w, k_stride=100, max_batch=8192, slots=2, route="batch",
                  min_batch=2048, max_wait_s=0.02, band_min=512)
    st2, (ids2, d2) = srv2.run(arr[:Rt], q[:Rt], ks[:Rt])
    assert st2["batches"] > 1
    assert (ids2 == rids[:Rt]).all() and (d2 == rd[:Rt]).all()
    assert np.isfinite(st2["p99_ms"])
