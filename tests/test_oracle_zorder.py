"""Pins of the oracle's Z-order key (the comparison curve of Sec. 2.2.1, whose
key intercalates the coordinates' bits) against what defines a Z-order
(Morton) curve rather than the oracle's own bit loop:

- the key is a bijection from the d-dim grid of m-bit coordinates onto the
  d*m-bit keys;
- two points compare at the most significant bit level where their
  coordinates differ, and within that level at the first dim that differs
  (the order of a trie over the levels; a pairwise rule, checked on random
  points with Python integers);
- the key never decreases when one coordinate grows (Morton order is monotone
  in every coordinate; a Hilbert curve is not);
- unlike the Hilbert curve it jumps: some consecutive keys are not
  neighbouring cells;
- at the index level, a window covering the whole list gives exact kNN, as
  with any curve.
"""
import itertools

import numpy as np
import pytest

MASK64 = (1 << 64) - 1


def all_cells(n, bits):
    side = 1 << bits
    return np.array(list(itertools.product(range(side), repeat=n)), np.uint32)


def keys_of(O, pts, bits):
    hi, lo = O.zorder_encode(pts, bits)
    return [O.key_int(a, b) for a, b in zip(hi, lo)]


def split(keys):
    return (np.array([k >> 64 for k in keys], np.uint64),
            np.array([k & MASK64 for k in keys], np.uint64))


SMALL = [(2, b) for b in range(1, 7)] + [(3, b) for b in range(1, 5)] + [(16, 1), (5, 2)]


@pytest.mark.parametrize("n,bits", SMALL)
def test_bijective_and_roundtrip(oracle, n, bits):
    pts = all_cells(n, bits)
    keys = keys_of(oracle, pts, bits)
    assert sorted(keys) == list(range(1 << (n * bits)))
    hi, lo = split(keys)
    assert (oracle.zorder_decode(hi, lo, n, bits) == pts).all()


def _trie_less(p, q, bits):
    """p before q: at the highest level where any coordinate differs, the first
    differing dim has bit 0 in p."""
    for lvl in range(bits - 1, -1, -1):
        for a, b in zip(p, q):
            ba, bb = (int(a) >> lvl) & 1, (int(b) >> lvl) & 1
            if ba != bb:
                return ba < bb
    return False


def test_pairwise_order_rule(oracle):
    rng = np.random.default_rng(5)
    pts = rng.integers(0, 256, size=(400, 16)).astype(np.uint32)
    pts[1] = pts[0]
    pts[2] = pts[0]
    pts[2, 15] ^= 1                         # differs only in the last bit of the last dim
    pts[3] = pts[0]
    pts[3, 0] ^= 128                        # differs only in the top bit of dim 0
    keys = keys_of(oracle, pts, 8)
    for i in range(0, 400, 3):
        for j in range(0, 400, 7):
            assert (keys[i] < keys[j]) == _trie_less(pts[i], pts[j], 8), (i, j)


@pytest.mark.parametrize("n,bits", [(2, 4), (3, 3)])
def test_monotone_in_every_coordinate(oracle, n, bits):
    pts = all_cells(n, bits)
    key = dict(zip(map(tuple, pts.tolist()), keys_of(oracle, pts, bits)))
    side = 1 << bits
    for p, kp in key.items():
        for d in range(n):
            if p[d] + 1 < side:
                q = list(p)
                q[d] += 1
                assert key[tuple(q)] > kp


def test_jumps_unlike_hilbert(oracle):
    n, bits = 2, 3
    total = 1 << (n * bits)
    hi, lo = split(range(total))
    z = oracle.zorder_decode(hi, lo, n, bits).astype(np.int64)
    h = oracle.hilbert_decode(hi, lo, n, bits).astype(np.int64)
    assert (np.abs(np.diff(h, axis=0)).sum(axis=1) == 1).all()
    assert (np.abs(np.diff(z, axis=0)).sum(axis=1) > 1).any()


def test_index_keys_and_full_window(oracle):
    rng = np.random.default_rng(8)
    db = rng.integers(0, 256, size=(700, 128), dtype=np.uint8)
    db[100:104] = db[5]
    q = rng.integers(0, 256, size=(30, 128), dtype=np.uint8)
    p = oracle.Params(curve="zorder")
    hi, lo = oracle.keys(db, p)
    # curve c's key is the Z-order key of dims 16c..16c+15
    for c in range(8):
        ehi, elo = oracle.zorder_encode(db[:, 16 * c:16 * c + 16], 8)
        assert (hi[:, c] == ehi).all() and (lo[:, c] == elo).all()
    ix = oracle.Index(db, p)
    for c in range(8):
        k = [oracle.key_int(a, b) for a, b in zip(ix.hi[c], ix.lo[c])]
        assert all(x <= y for x, y in zip(k, k[1:]))
    ids, d = ix.search(q, 10, 700)
    bi, bd = oracle.brute_force(db, q, 10)
    assert (ids == bi).all() and (d == bd).all()
    # and it differs from the Hilbert index
    hix = oracle.Index(db)
    assert not (hix.ids == ix.ids).all()
