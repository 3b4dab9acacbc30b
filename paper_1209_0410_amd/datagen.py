"""Seeded synthetic inputs shaped like the paper's SIFT workload.

The paper searches 128-d SIFT descriptors (Sec. 7: 130,463,526 database
vectors, 187,839 queries; experiments on a 1M subsample and on ~16.3M vectors
per node).  That set is not available here, so a seeded stand-in of the same
shape is used: 128 dims of uint8, non-negative and skewed toward 0, drawn from
a 64-component mixture.

Recipe (fixed, shared by the GPU library's tests and by the oracle's):
  centers C[64][128] ~ Exponential(scale 20) from default_rng(centers_seed);
  each row: z ~ U{0..63}, x = clip(rint(C[z] + N(0, 12^2)), 0, 255) as uint8
  (rint rounds half to even).
Rows are made in chunks of CHUNK rows; chunk j draws from
SeedSequence(seed, spawn_key=(j,)), so a smaller database is always a prefix of
a larger one with the same seed, and chunks can be generated in parallel.

This module holds random-number generation only: none of the method's
arithmetic lives here.
"""
from concurrent.futures import ThreadPoolExecutor
import os

import numpy as np

CHUNK = 65536
DIM = 128
COMPONENTS = 64

# Seeds of the standard workloads.
SEED_CENTERS = 0
SEED_DB = 1
SEED_QUERIES = 2
SEED_TRAIN = 3
SEED_EVAL = 4
SEED_CALIB = 5
SEED_UNEVEN = 6
SEED_ARRIVALS = 7


def centers(seed: int = SEED_CENTERS, dim: int = DIM) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.exponential(20.0, size=(COMPONENTS, dim))


def _chunk(seed: int, j: int, C: np.ndarray, rows: int) -> np.ndarray:
    rng = np.random.default_rng(np.random.SeedSequence(seed, spawn_key=(j,)))
    z = rng.integers(0, COMPONENTS, size=CHUNK)
    x = rng.normal(0.0, 12.0, size=(CHUNK, C.shape[1]))
    x += C[z]
    np.rint(x, out=x)
    np.clip(x, 0, 255, out=x)
    return x[:rows].astype(np.uint8)


def make_rows(n: int, seed: int, centers_seed: int = SEED_CENTERS, dim: int = DIM,
              out: np.ndarray = None, threads: int = None) -> np.ndarray:
    """n mixture rows (uint8, shape (n, dim)) for the given seed."""
    C = centers(centers_seed, dim)
    if out is None:
        out = np.empty((n, dim), np.uint8)
    nchunks = (n + CHUNK - 1) // CHUNK

    def work(j):
        lo = j * CHUNK
        take = min(CHUNK, n - lo)
        out[lo:lo + take] = _chunk(seed, j, C, take)

    if threads is None:
        threads = min(16, os.cpu_count() or 1)
    if nchunks <= 1 or threads <= 1:
        for j in range(nchunks):
            work(j)
    else:
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(work, range(nchunks)))
    return out


def make_db(n: int, seed: int = SEED_DB, **kw) -> np.ndarray:
    return make_rows(n, seed, **kw)


def make_queries(q: int, seed: int = SEED_QUERIES, **kw) -> np.ndarray:
    return make_rows(q, seed, **kw)


def uneven_w_k(q: int, seed: int = SEED_UNEVEN, w_lo: int = 8, w_hi: int = 512,
               ks=(1, 10, 100)):
    """Per-query probe depth, log-uniform in [w_lo, w_hi], and k drawn from ks."""
    rng = np.random.default_rng(seed)
    w = np.exp(rng.uniform(np.log(w_lo), np.log(w_hi), size=q))
    w = np.clip(np.rint(w), w_lo, w_hi).astype(np.uint32)
    k = rng.choice(np.asarray(ks, np.uint32), size=q)
    return w, k
