"""Pins of the oracle's index build and search (Alg. 1, Alg. 2, Eq. 2-3) against
library routines, brute force on tiny inputs and properties of the method:

- the lists are sorted by (key, id): numpy lexsort of the rows' keys agrees;
- the position is Python's bisect_left over (hi, lo) tuples;
- windows: w >= n makes every id a candidate; candidates grow with w; at most
  2w per curve; w = 1 takes exactly the neighbours on both sides of the place;
- distances and results: an independent numpy int64 brute force;
- with w covering the whole list the search is exact kNN (Eq. 3, ties by id);
- the label is the smallest w found by an explicit sweep.
"""
import bisect

import numpy as np
import pytest

from paper_1209_0410_amd import datagen


def np_brute(db, q, k):
    """Eq. (3) with ties broken by id, numpy int64."""
    d = ((q[:, None, :].astype(np.int64) - db[None, :, :].astype(np.int64)) ** 2).sum(-1)
    ids = np.zeros((q.shape[0], k), np.uint32)
    ds = np.zeros((q.shape[0], k), np.uint32)
    for i in range(q.shape[0]):
        order = np.lexsort((np.arange(db.shape[0]), d[i]))[:k]
        m = len(order)
        ids[i, :m], ds[i, :m] = order, d[i, order]
        ids[i, m:] = ds[i, m:] = 0xFFFFFFFF
    return ids, ds


def small_db(n, seed=1, dup_every=0):
    db = datagen.make_rows(n, seed)
    if dup_every:
        db[dup_every::dup_every] = db[0]
    return db


@pytest.fixture(scope="module")
def tiny(oracle):
    db = small_db(600, dup_every=97)          # forced duplicate rows and keys
    q = datagen.make_rows(40, 2)
    q[0] = db[5]                              # a query equal to a database row
    q[1] = 0                                  # key below (most of) the list
    q[2] = 255                                # key above (most of) the list
    return db, q, oracle.Index(db)


def key_tuples(ix, c):
    return list(zip(ix.hi[c].tolist(), ix.lo[c].tolist()))


def test_lists_sorted_by_key_then_id(oracle, tiny):
    db, _, ix = tiny
    hi, lo = oracle.keys(db, ix.p)
    for c in range(ix.p.curves):
        order = np.lexsort((np.arange(db.shape[0]), lo[:, c], hi[:, c]))
        assert (ix.ids[c] == order).all()
        assert (ix.hi[c] == hi[order, c]).all() and (ix.lo[c] == lo[order, c]).all()


def test_duplicate_keys_keep_id_order(oracle, tiny):
    db, _, ix = tiny
    for c in range(ix.p.curves):
        kt = key_tuples(ix, c)
        same = [i for i in range(1, len(kt)) if kt[i] == kt[i - 1]]
        assert same, "the fixture forces repeated keys"
        assert all(ix.ids[c][i] > ix.ids[c][i - 1] for i in same)


def test_positions_are_bisect_left(oracle, tiny):
    db, q, ix = tiny
    pos = ix.positions(q)
    qhi, qlo = oracle.keys(q, ix.p)
    for c in range(ix.p.curves):
        kt = key_tuples(ix, c)
        for i in range(q.shape[0]):
            want = bisect.bisect_left(kt, (int(qhi[i, c]), int(qlo[i, c])))
            assert pos[i, c] == want
            assert oracle.lower_bound(ix.hi[c], ix.lo[c], qhi[i, c], qlo[i, c]) == want


def test_window_w1_takes_both_neighbours(oracle, tiny):
    db, q, ix = tiny
    pos = ix.positions(q)
    cand = ix.candidates(q, 1)
    n = db.shape[0]
    for i in range(q.shape[0]):
        want = set()
        for c in range(ix.p.curves):
            p = int(pos[i, c])
            if p > 0:
                want.add(int(ix.ids[c][p - 1]))      # last key < qkey
            if p < n:
                want.add(int(ix.ids[c][p]))          # first key >= qkey
        assert set(cand[i].tolist()) == want


def test_candidates_monotone_bounded_and_complete(oracle, tiny):
    db, q, ix = tiny
    n = db.shape[0]
    prev = None
    for w in [0, 1, 2, 3, 5, 8, 13, 40, 150, 299, 300, 600, 10_000]:
        cand = ix.candidates(q, w)
        for i, cset in enumerate(cand):
            assert (np.diff(cset.astype(np.int64)) > 0).all()       # sorted, distinct
            assert len(cset) <= min(n, 2 * w * ix.p.curves)
            if prev is not None:
                assert set(prev[i].tolist()) <= set(cset.tolist())
            if w >= n:
                assert len(cset) == n
        prev = cand


def test_brute_force_matches_numpy(oracle, tiny):
    db, q, _ = tiny
    for k in [1, 10, 37]:
        ids, d = oracle.brute_force(db, q, k)
        rid, rd = np_brute(db, q, k)
        assert (ids == rid).all() and (d == rd).all()


def test_search_distances_match_numpy(oracle, tiny):
    db, q, ix = tiny
    ids, d = ix.search(q, 100, 4)
    for i in range(q.shape[0]):
        m = ids[i] != 0xFFFFFFFF
        ref = ((db[ids[i, m]].astype(np.int64) - q[i].astype(np.int64)) ** 2).sum(-1)
        assert (d[i, m] == ref).all()
        keys = list(zip(d[i, m].tolist(), ids[i, m].tolist()))
        assert keys == sorted(keys)


def test_search_with_full_window_is_exact_knn(oracle, tiny):
    db, q, ix = tiny
    for k in [1, 10, 100]:
        ids, d = ix.search(q, k, db.shape[0])
        rid, rd = np_brute(db, q, k)
        assert (ids == rid).all() and (d == rd).all()


def test_search_is_top_k_of_candidates(oracle, tiny):
    db, q, ix = tiny
    for w in [1, 3, 16]:
        cand = ix.candidates(q, w)
        ids, d = ix.search(q, 10, w)
        for i in range(q.shape[0]):
            c = cand[i].astype(np.int64)
            dist = ((db[c].astype(np.int64) - q[i].astype(np.int64)) ** 2).sum(-1)
            order = np.lexsort((c, dist))[:10]
            m = len(order)
            assert (ids[i, :m] == c[order]).all() and (d[i, :m] == dist[order]).all()
            assert (ids[i, m:] == 0xFFFFFFFF).all() and (d[i, m:] == 0xFFFFFFFF).all()


def test_query_equal_to_row_finds_it(oracle, tiny):
    db, q, ix = tiny
    ids, d = ix.search(q[:1], 1, 1)
    assert d[0, 0] == 0 and (db[ids[0, 0]] == q[0]).all()


def test_fewer_rows_than_k_pads(oracle):
    db = small_db(7)
    q = datagen.make_rows(5, 3)
    ix = oracle.Index(db)
    ids, d = ix.search(q, 10, 1000)
    rid, rd = np_brute(db, q, 10)
    assert (ids == rid).all() and (d == rd).all()
    assert (ids[:, 7:] == 0xFFFFFFFF).all()


def test_single_row_database(oracle):
    db = small_db(1)
    q = datagen.make_rows(3, 3)
    ix = oracle.Index(db)
    for w in [0, 1, 5]:
        ids, d = ix.search(q, 2, w)
        if w == 0:
            assert (ids == 0xFFFFFFFF).all()
        else:
            assert (ids[:, 0] == 0).all() and (ids[:, 1] == 0xFFFFFFFF).all()


def test_permutation_changes_keys_not_exactness(oracle):
    db = small_db(300)
    q = datagen.make_rows(10, 2)
    perm = np.random.default_rng(5).permutation(128)
    ix = oracle.Index(db, oracle.Params(perm=perm))
    hi, lo = oracle.keys(db[:4], ix.p)
    proj = db[:4][:, perm[:16]].astype(np.uint32)
    h0, l0 = oracle.hilbert_encode(proj, 8)
    assert (hi[:, 0] == h0).all() and (lo[:, 0] == l0).all()
    ids, d = ix.search(q, 5, 300)
    rid, rd = np_brute(db, q, 5)
    assert (ids == rid).all() and (d == rd).all()


def test_label_is_smallest_recovering_window(oracle, tiny):
    db, q, ix = tiny
    for k in [1, 5]:
        truth, _ = oracle.brute_force(db, q, k)
        lab = ix.labels(q, k, truth)
        for i in range(q.shape[0]):
            w = 0
            while True:
                ids, _ = ix.search(q[i:i + 1], k, w)
                if (ids[0] == truth[i]).all():
                    break
                w += 1
            assert lab[i] == w


def test_features_special_cases(oracle, tiny):
    db, q, ix = tiny
    f = ix.features(q, 10)
    assert f.shape == (q.shape[0], 24)
    assert np.allclose(f[:, 20], np.log2(10))
    # q[0] equals row 5: at its place in every list sits an entry with its key,
    # so the gap to the first entry >= qkey is 0 (both min and mean).
    assert f[0, 3] == 0.0 and f[0, 9] == 0.0
    pos = ix.positions(q[:1])
    for c in range(8):
        row = db[ix.ids[c][pos[0, c]]]
        d = int(((row.astype(np.int64) - q[0].astype(np.int64)) ** 2).sum())
        assert f[0, 12 + c] == pytest.approx(np.log2(1 + d))
    # the key gaps are ordered: min <= mean, and wider spans never shrink
    assert (f[:, 0:6] <= f[:, 6:12] + 1e-12).all()
    assert (f[:, 21] <= f[:, 22] + 1e-12).all() and (f[:, 22] <= f[:, 23] + 1e-12).all()


def test_features_match_python_bigint(oracle, tiny):
    db, q, ix = tiny
    f = ix.features(q, 7)
    pos = ix.positions(q)
    qhi, qlo = oracle.keys(q, ix.p)
    n = db.shape[0]
    cl = lambda v: min(max(v, 0), n - 1)
    K = lambda c, i: (int(ix.hi[c][i]) << 64) | int(ix.lo[c][i])
    for i in range(q.shape[0]):
        qk = [(int(qhi[i, c]) << 64) | int(qlo[i, c]) for c in range(8)]
        for j, o in enumerate([-64, -8, -1, 1, 8, 64]):
            g = [np.log2(1.0 + float(abs(K(c, cl(pos[i, c] + (o if o < 0 else o - 1))) - qk[c])))
                 for c in range(8)]
            assert f[i, j] == pytest.approx(min(g), rel=1e-12)
            assert f[i, 6 + j] == pytest.approx(np.mean(g), rel=1e-12)
        for j, s in enumerate([1, 8, 64]):
            g = [np.log2(1.0 + float(K(c, cl(pos[i, c] + s - 1)) - K(c, cl(pos[i, c] - s))))
                 for c in range(8)]
            assert f[i, 21 + j] == pytest.approx(max(g), rel=1e-12)


def _hand_built_index(oracle, key_of_entry, n):
    """An oracle index whose lists are written by hand: curve c's entry i has
    key key_of_entry(c, i) (integers, ascending in i) and id (i - 100 + c) mod n
    (so entry 100 of curve c holds id c).  The query's subspace of curve c is
    the point the Hilbert decode gives for key 100 (c + 1), so its key there is
    exactly that integer.  Database row j < 8 is the query with dim 127 raised
    by j + 1 (squared distance (j + 1)^2); the other rows are far."""
    p = oracle.Params()
    q = np.zeros(128, np.uint8)
    for c in range(8):
        pt = oracle.hilbert_decode(np.array([0], np.uint64),
                                   np.array([100 * (c + 1)], np.uint64), 16, 8)[0]
        q[16 * c:16 * c + 16] = pt
    hi, lo = oracle.keys(q[None], p)
    assert all(oracle.key_int(hi[0, c], lo[0, c]) == 100 * (c + 1) for c in range(8))
    db = np.tile(q, (n, 1))
    db[:, 0] = np.minimum(db[:, 0].astype(np.int64) + 60, 255).astype(np.uint8)
    for j in range(8):
        db[j] = q
        db[j, 127] = q[127] + j + 1
    ix = oracle.Index.__new__(oracle.Index)
    ix.p, ix.db, ix.n = p, np.ascontiguousarray(db), n
    ix.hi = np.zeros((8, n), np.uint64)
    ix.lo = np.zeros((8, n), np.uint64)
    ix.ids = np.zeros((8, n), np.uint32)
    for c in range(8):
        for i in range(n):
            kv = key_of_entry(c, i)
            ix.hi[c, i] = kv >> 64
            ix.lo[c, i] = kv & ((1 << 64) - 1)
            ix.ids[c, i] = (i - 100 + c) % n
    return ix, q


def test_features_hand_built_interior(oracle):
    """Curve c's keys are (c + 1) * i for i = 0..n-1 (curve 0: the integers
    0..n-1); the query's key is 100 (c + 1), so its place is 100 on every curve.
    The expected 24 features are written out from that construction, not from
    the feature formulas."""
    n = 200
    ix, q = _hand_built_index(oracle, lambda c, i: (c + 1) * i, n)
    assert (ix.positions(q[None]) == 100).all()
    f = ix.features(q[None], 10)[0]
    L = np.log2
    cs = np.arange(1, 9)
    # key gaps to the entries at offsets -64, -8, -1 and +1, +8, +64, which sit
    # 64, 8, 1, 0, 7 and 63 entries from the place: gap = (c + 1) * that
    expect_min = [L(65), L(9), L(2), 0.0, L(8), L(64)]
    expect_mean = [np.mean(L(1 + cs * d)) for d in (64, 8, 1, 0, 7, 63)]
    # first candidates: row c, at squared distance (c + 1)^2
    expect_first = list(L(1 + cs ** 2))
    # spans: entries pos - s .. pos + s - 1 cover 2s - 1 steps; the widest
    # curve (spacing 8) gives the max
    expect_span = [L(1 + 8 * 1), L(1 + 8 * 15), L(1 + 8 * 127)]
    expect = expect_min + expect_mean + expect_first + [L(10)] + expect_span
    assert f.shape == (24,)
    assert np.allclose(f, expect, rtol=0, atol=1e-12), (f, expect)


def test_features_hand_built_list_start(oracle):
    """Keys (c + 1) (i + 1) + 100 (c + 1): every key is above the query's, so its
    place is 0 and the entries before it clamp to entry 0."""
    n = 200
    ix, q = _hand_built_index(oracle, lambda c, i: (c + 1) * (i + 1) + 100 * (c + 1), n)
    assert (ix.positions(q[None]) == 0).all()
    f = ix.features(q[None], 1)[0]
    L = np.log2
    cs = np.arange(1, 9)
    # entries at -64, -8, -1 and +1 all clamp to or are entry 0 (gap c + 1);
    # +8 is entry 7 (gap 8 (c + 1)), +64 is entry 63 (gap 64 (c + 1))
    steps = (1, 1, 1, 1, 8, 64)
    expect_min = [L(1 + s) for s in steps]
    expect_mean = [np.mean(L(1 + cs * s)) for s in steps]
    # entry 0 of curve c holds id (c - 100) mod n, one of the far rows: query
    # plus 60 in dim 0
    expect_first = [L(1 + 60 ** 2)] * 8
    # spans: entry s - 1 minus entry 0 (the lower end clamps): (c + 1)(s - 1)
    expect_span = [0.0, L(1 + 8 * 7), L(1 + 8 * 63)]
    expect = expect_min + expect_mean + expect_first + [0.0] + expect_span
    assert np.allclose(f, expect, rtol=0, atol=1e-12), (f, expect)
