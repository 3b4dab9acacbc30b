"""GPU parity at full size: N = 10^7 rows, a batch of Q = 10^5 queries, k = 10,
launched exactly as the timed step is (keys encoded into the scratch, then the
search with the path chosen automatically: the banded kernel over the row
store at the recall-0.90 window, the gather kernel at small windows).  The
oracle cannot search the whole batch in seconds, so it searches a sample of
queries spread over the batch, one by one; those rows must match bit for bit
(Alg. 2 with Eq. (2) distances, results ordered by (distance, id))."""
import numpy as np
import pytest

from conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

N, Q, K = 10_000_000, 100_000, 10
W_RECALL90 = 27_648          # fixed window that reaches recall@10 >= 0.90 on this recipe
PATH_GATHER, PATH_BAND = 1, 2


def u32(t):
    return t.cpu().numpy().view(np.uint32)


@pytest.fixture(scope="module")
def full(oracle):
    import torch
    from paper_1209_0410_amd import datagen
    from paper_1209_0410_amd.index import Index
    db = datagen.make_db(N)
    q = datagen.make_queries(Q)
    dev = torch.device("cuda:0")
    print(f"[full] building GPU index and row store n={N}", flush=True)
    gdb = torch.from_numpy(db).to(dev)
    gq = torch.from_numpy(q).to(dev)
    gix = Index(gdb)
    gix.attach_rowstore()
    sc = gix.scratch(Q)
    out = (torch.empty((Q, K), dtype=torch.int32, device=dev),
           torch.empty((Q, K), dtype=torch.int32, device=dev))
    print("[full] building oracle index", flush=True)
    oix = oracle.Index(db)
    # spread over the batch (first, last, and evenly between) plus a few at random
    rng = np.random.default_rng(1209)
    pick = np.unique(np.concatenate([np.linspace(0, Q - 1, 96).astype(np.int64),
                                     rng.integers(0, Q, size=32)]))
    yield dict(q=q, gq=gq, gix=gix, sc=sc, out=out, oix=oix, pick=pick)
    gix.detach_rowstore()


@pytest.mark.parametrize("w,path,k", [(W_RECALL90, PATH_BAND, K), (64, PATH_GATHER, K),
                                      (4096, PATH_BAND, K), (W_RECALL90, PATH_BAND, 1),
                                      (W_RECALL90, PATH_BAND, 16), (64, PATH_GATHER, 100)])
def test_full_size_sampled_rows_bit_exact(full, w, path, k):
    import torch
    gix, sc = full["gix"], full["sc"]
    out = full["out"] if k == K else tuple(
        torch.empty((Q, k), dtype=torch.int32, device=full["gq"].device) for _ in range(2))
    assert gix.path(Q, k, w, sc.numel()) == path
    print(f"[full] w={w} path={path} k={k} on {len(full['pick'])} sampled queries", flush=True)
    out[0].fill_(0)
    out[1].fill_(0)
    gix.encode_queries(full["gq"], sc)
    gix.search_encoded(full["gq"], k, w, out, sc)
    ids, d = u32(out[0]), u32(out[1])
    pick = full["pick"]
    rid, rd = full["oix"].search(full["q"][pick], k, w)
    assert (ids[pick] == rid).all() and (d[pick] == rd).all()
    # every row of the batch, sampled or not: ascending by (distance, id), no
    # repeated id, all slots filled (every window holds more than k rows)
    key = (d.astype(np.uint64) << np.uint64(32)) | ids.astype(np.uint64)
    assert (key[:, 1:] > key[:, :-1]).all()
    assert (ids < N).all()


@pytest.mark.parametrize("k", [17, 100])
def test_full_size_band_two_pass_sampled_rows_bit_exact(full, k):
    """k > 16 on the banded path at full size (two passes over the row store,
    the scratch sized for that k), launched as the timed step is."""
    import torch
    gix = full["gix"]
    sc = gix.new_scratch(Q, k)
    out = tuple(torch.empty((Q, k), dtype=torch.int32, device=full["gq"].device)
                for _ in range(2))
    assert gix.path(Q, k, W_RECALL90, sc.numel()) == PATH_BAND
    print(f"[full] k={k} banded two passes on {len(full['pick'])} sampled queries", flush=True)
    gix.encode_queries(full["gq"], sc)
    gix.search_encoded(full["gq"], k, W_RECALL90, out, sc)
    ids, d = u32(out[0]), u32(out[1])
    del sc
    pick = full["pick"]
    rid, rd = full["oix"].search(full["q"][pick], k, W_RECALL90)
    assert (ids[pick] == rid).all() and (d[pick] == rd).all()
    key = (d.astype(np.uint64) << np.uint64(32)) | ids.astype(np.uint64)
    assert (key[:, 1:] > key[:, :-1]).all()
    assert (ids < N).all()


def test_full_size_per_query_w_sampled_rows_bit_exact(full):
    """The learned step's launch: a w per query (here log-uniform over the
    spread the learned model gives at recall 0.90) on the banded path."""
    import torch
    gix, sc, out = full["gix"], full["sc"], full["out"]
    rng = np.random.default_rng(1210)
    w = np.exp(rng.uniform(np.log(16_384), np.log(65_536), size=Q)).astype(np.uint32)
    gw = torch.from_numpy(w.view(np.int32)).to(full["gq"].device)
    assert gix.path(Q, K, int(w.max()), sc.numel()) == PATH_BAND
    print(f"[full] per-query w in [{w.min()}, {w.max()}]", flush=True)
    out[0].fill_(0)
    out[1].fill_(0)
    gix.encode_queries(full["gq"], sc)
    gix.search_encoded(full["gq"], K, int(w.max()), out, sc, w_per_query=gw)
    ids, d = u32(out[0]), u32(out[1])
    pick = full["pick"]
    rid, rd = full["oix"].search(full["q"][pick], K, w[pick])
    assert (ids[pick] == rid).all() and (d[pick] == rd).all()


def test_full_size_uneven_batch_sampled_rows_bit_exact(full):
    """The uneven step's launch: 2 x 10^5 queries, w log-uniform in [8, 512] and
    k from {1, 10, 100} per query, the autotuned shape, captured in a HIP graph
    and replayed; row q holds its k_q results, then empty slots."""
    import torch
    from paper_1209_0410_amd import datagen
    from paper_1209_0410_amd.tune import Graph, Tuner
    gix = full["gix"]
    nq = 200_000
    q = datagen.make_queries(nq, seed=datagen.SEED_UNEVEN)
    w, k = datagen.uneven_w_k(nq)
    dev = full["gq"].device
    gq = torch.from_numpy(q).to(dev)
    gw = torch.from_numpy(w.view(np.int32)).to(dev)
    gk = torch.from_numpy(k.view(np.int32)).to(dev)
    kst = int(k.max())
    cfg, entry = Tuner().best(gix, gq, gw, gk, sample=nq)
    print(f"[full] uneven shape chunk={cfg.chunk_slots} split={cfg.max_split} "
          f"per_cu={cfg.blocks_per_cu}", flush=True)
    sc = gix.uneven_scratch(nq, kst, cfg)
    out = (torch.zeros((nq, kst), dtype=torch.int32, device=dev),
           torch.zeros((nq, kst), dtype=torch.int32, device=dev))
    g = Graph(lambda: gix.search_uneven(gq, w_per_query=gw, k_per_query=gk, k_stride=kst,
                                        cfg=cfg, out=out, scratch=sc))
    rng = np.random.default_rng(1211)
    pick = np.unique(np.concatenate([np.linspace(0, nq - 1, 256).astype(np.int64),
                                     rng.integers(0, nq, size=64)]))
    for rep in range(2):
        g.replay()
        torch.cuda.synchronize()
        ids, d = u32(out[0]), u32(out[1])
        for kk in np.unique(k[pick]):
            sel = pick[k[pick] == kk]
            rid, rd = full["oix"].search(q[sel], int(kk), w[sel])
            assert (ids[sel, :kk] == rid).all() and (d[sel, :kk] == rd).all(), (rep, kk)
            assert (ids[sel, kk:] == 0xFFFFFFFF).all() and (d[sel, kk:] == 0xFFFFFFFF).all()
        out[0].fill_(0)
        out[1].fill_(0)
