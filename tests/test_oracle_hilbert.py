"""Pins of the oracle's Hilbert extended key (Sec. 2.2.1) against what the
mathematics fixes, independent of the oracle's own formulas:

- C^-1 is a bijection from the d-dim grid of m-bit coordinates onto the
  d*m-bit keys (the paper: every finite order of the curve is bijective and
  keeps the number of bits);
- consecutive keys are neighbouring grid cells (L1 distance 1), the defining
  property of a Hilbert curve;
- every aligned block of 2^(d*l) consecutive keys fills an aligned sub-cube of
  side 2^l (the recursive construction);
- d = 1 gives the identity or the reversal, the only unit-step orders of a line;
- d = 2 is the classic curve (golden fixture) up to the symmetries of the
  square and reversal.
"""
import itertools
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
MASK64 = (1 << 64) - 1


def split(keys):
    hi = np.array([k >> 64 for k in keys], np.uint64)
    lo = np.array([k & MASK64 for k in keys], np.uint64)
    return hi, lo


def all_cells(n, bits):
    side = 1 << bits
    return np.array(list(itertools.product(range(side), repeat=n)), np.uint32)


def keys_of(O, pts, bits):
    hi, lo = O.hilbert_encode(pts, bits)
    return [O.key_int(a, b) for a, b in zip(hi, lo)]


SMALL = [(2, b) for b in range(1, 7)] + [(3, b) for b in range(1, 5)] + [(4, 4), (16, 1),
                                                                          (5, 2), (1, 6)]


@pytest.mark.parametrize("n,bits", SMALL)
def test_bijective_small_grids(oracle, n, bits):
    pts = all_cells(n, bits)
    keys = keys_of(oracle, pts, bits)
    assert sorted(keys) == list(range(1 << (n * bits)))


@pytest.mark.parametrize("n,bits", SMALL)
def test_adjacency_and_roundtrip_small_grids(oracle, n, bits):
    total = 1 << (n * bits)
    hi, lo = split(range(total))
    cells = oracle.hilbert_decode(hi, lo, n, bits).astype(np.int64)
    assert cells.max() < (1 << bits)
    steps = np.abs(np.diff(cells, axis=0)).sum(axis=1)
    assert (steps == 1).all()
    back = keys_of(oracle, cells.astype(np.uint32), bits)
    assert back == list(range(total))


@pytest.mark.parametrize("n,bits", [(2, 5), (3, 4), (4, 3)])
def test_blocks_fill_subcubes(oracle, n, bits):
    total = 1 << (n * bits)
    hi, lo = split(range(total))
    cells = oracle.hilbert_decode(hi, lo, n, bits).astype(np.int64)
    for lvl in range(1, bits):
        blk = 1 << (n * lvl)
        side = 1 << lvl
        for j in range(total // blk):
            c = cells[j * blk:(j + 1) * blk]
            lo_c = c.min(axis=0)
            assert (lo_c % side == 0).all()
            assert (c.max(axis=0) - lo_c == side - 1).all()


def test_decode_zero_is_origin(oracle):
    for n, bits in [(2, 3), (16, 8), (7, 5)]:
        z = np.zeros(1, np.uint64)
        assert (oracle.hilbert_decode(z, z, n, bits) == 0).all()


def test_d1_is_identity_or_reversal(oracle):
    for bits in range(1, 9):
        pts = np.arange(1 << bits, dtype=np.uint32)[:, None]
        keys = keys_of(oracle, pts, bits)
        ident = list(range(1 << bits))
        assert keys == ident or keys == ident[::-1]


def _golden_2d():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "hilbert2d_order2.txt"))
            if l.strip() and not l.startswith("#")]
    return np.array(rows, np.int64)


def _classic_2d(order):
    """Textbook rotate/reflect construction of the 2-D Hilbert curve."""
    side = 1 << order
    out = []
    for d in range(side * side):
        x = y = 0
        t = d
        s = 1
        while s < side:
            rx = 1 & (t // 2)
            ry = 1 & (t ^ rx)
            if ry == 0:
                if rx == 1:
                    x, y = s - 1 - x, s - 1 - y
                x, y = y, x
            x += s * rx
            y += s * ry
            t //= 4
            s *= 2
        out.append((x, y))
    return np.array(out, np.int64)


def _symmetries(path, side):
    m = side - 1
    for swap in (False, True):
        for fx in (False, True):
            for fy in (False, True):
                p = path[:, ::-1] if swap else path.copy()
                if fx:
                    p[:, 0] = m - p[:, 0]
                if fy:
                    p[:, 1] = m - p[:, 1]
                yield p
                yield p[::-1]


def test_classic_construction_matches_golden():
    gold = _golden_2d()
    assert any((s == gold).all() for s in _symmetries(_classic_2d(2), 4))


@pytest.mark.parametrize("order", [1, 2, 3, 4, 5])
def test_d2_is_classic_hilbert_up_to_symmetry(oracle, order):
    total = 1 << (2 * order)
    hi, lo = split(range(total))
    ours = oracle.hilbert_decode(hi, lo, 2, order).astype(np.int64)
    ref = _classic_2d(order)
    assert any((s == ours).all() for s in _symmetries(ref, 1 << order))


def test_full_size_random_adjacency_and_roundtrip(oracle):
    """d = 16, m = 8 (the 128-bit keys of the search): 10^6 random keys."""
    rng = np.random.default_rng(11)
    m = 1_000_000
    hi = rng.integers(0, 1 << 63, size=m, dtype=np.uint64) * 2 + rng.integers(0, 2, size=m,
                                                                             dtype=np.uint64)
    lo = rng.integers(0, 1 << 63, size=m, dtype=np.uint64) * 2 + rng.integers(0, 2, size=m,
                                                                             dtype=np.uint64)
    ok = ~((hi == np.uint64(MASK64)) & (lo == np.uint64(MASK64)))
    hi, lo = hi[ok], lo[ok]
    lo1 = lo + np.uint64(1)
    hi1 = hi + (lo1 == 0).astype(np.uint64)
    a = oracle.hilbert_decode(hi, lo, 16, 8).astype(np.int64)
    b = oracle.hilbert_decode(hi1, lo1, 16, 8).astype(np.int64)
    assert (np.abs(a - b).sum(axis=1) == 1).all()
    h2, l2 = oracle.hilbert_encode(a.astype(np.uint32), 8)
    assert (h2 == hi).all() and (l2 == lo).all()


def test_full_size_subcube_nesting(oracle):
    """The top 16*l bits of a 128-bit key name an aligned sub-cube of side 2^(8-l)."""
    rng = np.random.default_rng(12)
    for _ in range(20):
        lvl_keep = int(rng.integers(1, 8))          # levels fixed by the prefix
        free = 16 * (8 - lvl_keep)                  # free low bits
        prefix = int(rng.integers(0, 1 << 62)) << 66 >> (128 - 16 * lvl_keep) << free
        offs = rng.integers(0, 1 << min(free, 62), size=2000)
        keys = [prefix | int(o) for o in offs] + [prefix, prefix | ((1 << free) - 1)]
        hi, lo = split(keys)
        cells = oracle.hilbert_decode(hi, lo, 16, 8).astype(np.int64)
        side = 1 << (8 - lvl_keep)
        corner = cells.min(axis=0) // side * side
        assert (cells // side == corner // side).all()
