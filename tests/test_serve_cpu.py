"""Host-side parts of the request loop (no GPU): the seeded arrival process,
the batch route's unpacking and the blocks of the device-memory budget."""
import numpy as np


def test_arrivals_follow_the_rate():
    from paper_1209_0410_amd.serve import sinusoidal_arrivals
    t = sinusoidal_arrivals(60.0, 1000, 20000, 60.0, seed=7)
    assert (np.diff(t) >= 0).all() and t.min() >= 0 and t.max() <= 60
    # expected count = mean rate x duration = 10,500 x 60
    assert abs(len(t) - 630_000) < 5 * np.sqrt(630_000)
    # the rate is lowest at the ends of the period and highest in the middle
    c = np.histogram(t, bins=6, range=(0, 60))[0]
    assert c[2] > 3 * c[0] and c[3] > 3 * c[5]


def test_batch_route_unpacks_k_classes():
    """The batch route's host side: a batch packed by k (stable), each class's
    results in a compact [count x k] block, all ids then all distances; the
    unpacking puts every request's k results back in its row and pads the
    row with 0xFFFFFFFF."""
    import types
    import torch
    from paper_1209_0410_amd.serve import Server
    rng = np.random.default_rng(5)
    lo, nq, k_stride = 7, 50, 100
    ks = rng.choice([1, 10, 100], size=lo + nq).astype(np.uint32)
    perm = np.argsort(ks[lo:], kind="stable")
    kp = ks[lo:][perm]
    classes, o = [], 0
    for kv in np.unique(kp):
        m = int((kp == kv).sum())
        classes.append((int(kv), o, m))
        o += m
    tot = sum(kv * m for kv, _, m in classes)
    # the device's blocks: request r's j-th result has id 1000 r + j, distance r + j
    ids, dists, off = np.zeros(tot, np.uint32), np.zeros(tot, np.uint32), 0
    for kv, first, m in classes:
        for i in range(m):
            r = lo + perm[first + i]
            ids[off + i * kv: off + (i + 1) * kv] = 1000 * r + np.arange(kv)
            dists[off + i * kv: off + (i + 1) * kv] = r + np.arange(kv)
        off += m * kv
    h = torch.from_numpy(np.concatenate([ids, dists]).view(np.int32).copy())
    slot = types.SimpleNamespace(h_out=h, classes=classes, perm=perm, tot=tot)
    srv = Server.__new__(Server)
    res_i = np.zeros((lo + nq, k_stride), np.uint32)
    res_d = np.zeros((lo + nq, k_stride), np.uint32)
    srv._unpack(slot, lo, lo + nq, res_i, res_d)
    for r in range(lo, lo + nq):
        kv = int(ks[r])
        assert (res_i[r, :kv] == 1000 * r + np.arange(kv)).all()
        assert (res_d[r, :kv] == r + np.arange(kv)).all()
        assert (res_i[r, kv:] == 0xFFFFFFFF).all() and (res_d[r, kv:] == 0xFFFFFFFF).all()
    assert (res_i[:lo] == 0).all()


def test_budget_blocks_first_fit_and_merge():
    """The serving budget hands out 256-byte-aligned blocks of one buffer,
    first fit, and merges returned blocks with free neighbours."""
    import torch
    from paper_1209_0410_amd.serve import HbmBudget
    b = HbmBudget(4096 + 100).bind(torch.device("cpu"), 1 << 20)
    assert b.budget == 4096 and b.buf.numel() == 4096 and b.buf.data_ptr() % 256 == 0
    a = b.take(1000)                        # 1024 bytes
    c = b.take(1024)
    d = b.take(2048)
    assert (a, c, d) == (0, 1024, 2048) and b.used == 4096 and b.largest() == 0
    assert b.take(1) is None
    b.give(c, 1024)
    assert b.largest() == 1024 and b.take(1025) is None
    b.give(a, 1000)                         # merges with the block at 1024
    assert b.largest() == 2048 and b.take(2048) == 0
    b.give(0, 2048)
    b.give(d, 2048)
    assert b.used == 0 and b.largest() == 4096 and b.peak == 4096
    assert HbmBudget(1 << 30).bind(torch.device("cpu"), 5000).budget == 5120
