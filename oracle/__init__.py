"""CPU oracle for the Multicurves search path (numpy front end over hc_oracle.c).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark are its only callers.  The GPU library never imports it,
and it imports nothing from the GPU package.

Arrays are numpy; index lists are laid out [curve][n]; per-query keys and
positions are laid out [query][curve].  See hc_oracle.c for the passages of
the paper each routine follows.
"""
import ctypes as ct
import os

import numpy as np

from . import build as _build

_LIB = None

_u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")
_u16p = np.ctypeslib.ndpointer(np.uint16, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
_u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_i64 = ct.c_int64
_int = ct.c_int
_dbl = ct.c_double

_SIGS = {
    "hco_hilbert_encode": [_u32p, _i64, _int, _int, _u64p, _u64p],
    "hco_hilbert_decode": [_u64p, _u64p, _i64, _int, _int, _u32p],
    "hco_zorder_encode": [_u32p, _i64, _int, _int, _u64p, _u64p],
    "hco_zorder_decode": [_u64p, _u64p, _i64, _int, _int, _u32p],
    "hco_keys_ex": [_u8p, _i64, _int, _u16p, _int, _int, _int, _int, _u64p, _u64p],
    "hco_build_ex": [_u8p, _i64, _int, _u16p, _int, _int, _int, _int, _u64p, _u64p, _u32p],
    "hco_positions": [_u64p, _u64p, _i64, _int, _u16p, _int, _int, _int, _int, _u8p, _i64,
                      _i64p],
    "hco_candidates": [_u64p, _u64p, _u32p, _i64, _int, _u16p, _int, _int, _int, _int,
                       _u8p, _i64, _u32p, _u32p, _u32p, _i64],
    "hco_search": [_u64p, _u64p, _u32p, _u8p, _i64, _int, _u16p, _int, _int, _int, _int,
                   _u8p, _i64, _int, _u32p, _u32p, _u32p],
    "hco_brute_force": [_u8p, _i64, _int, _u8p, _i64, _int, _u32p, _u32p],
    "hco_labels": [_u64p, _u64p, _u32p, _i64, _int, _u16p, _int, _int, _int, _int, _u8p,
                   _i64, _int, _u32p, _u32p],
    "hco_features": [_u64p, _u64p, _u32p, _u8p, _i64, _int, _u16p, _int, _int, _int, _int,
                     _u8p, _i64, _u32p, _f64p],
    "hco_mlp_forward": [_f64p, _f64p, _i64, _int, _int, _int, _f64p],
    "hco_mlp_loss_grad": [_f64p, _f64p, _f64p, _i64, _int, _int, _int, _f64p,
                          ct.POINTER(ct.c_double)],
    "hco_adam_step": [_f64p, _f64p, _f64p, _f64p, _i64, _i64, _dbl, _dbl, _dbl, _dbl],
}


def lib():
    """Load (building on first use if needed) the oracle shared library."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ct.CDLL(_build.lib_path())
        for name, args in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ct.c_int
        L.hco_lower_bound.argtypes = [_u64p, _u64p, _i64, ct.c_uint64, ct.c_uint64]
        L.hco_lower_bound.restype = ct.c_int64
        L.hco_mlp_nparams.argtypes = [_int, _int, _int]
        L.hco_mlp_nparams.restype = ct.c_int64
        L.hco_set_threads.argtypes = [_int]
        L.hco_set_threads.restype = None
        L.hco_threads.argtypes = []
        L.hco_threads.restype = _int
        _LIB = L
    return _LIB


def set_threads(t):
    """Threads of the oracle's parallel loops from now on (t >= 1)."""
    lib().hco_set_threads(int(t))


def threads():
    """Threads the oracle's parallel loops use."""
    return int(lib().hco_threads())


def _check(rc, name):
    if rc != 0:
        raise RuntimeError(f"oracle {name} failed with status {rc}")


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


# ---------------------------------------------------------------------------
# Hilbert extended key (Sec. 2.2.1)
# ---------------------------------------------------------------------------

def hilbert_encode(coords, bits):
    """coords: (P, n) uint -> (hi, lo) uint64 arrays of the order-`bits` key."""
    c = _c(coords, np.uint32)
    P, n = c.shape
    hi = np.zeros(P, np.uint64)
    lo = np.zeros(P, np.uint64)
    _check(lib().hco_hilbert_encode(c, P, n, bits, hi, lo), "hilbert_encode")
    return hi, lo


def hilbert_decode(hi, lo, n, bits):
    hi = _c(hi, np.uint64)
    lo = _c(lo, np.uint64)
    out = np.zeros((hi.shape[0], n), np.uint32)
    _check(lib().hco_hilbert_decode(hi, lo, hi.shape[0], n, bits, out), "hilbert_decode")
    return out


def zorder_encode(coords, bits):
    """coords: (P, n) uint -> (hi, lo) uint64 arrays of the Z-order key."""
    c = _c(coords, np.uint32)
    P, n = c.shape
    hi = np.zeros(P, np.uint64)
    lo = np.zeros(P, np.uint64)
    _check(lib().hco_zorder_encode(c, P, n, bits, hi, lo), "zorder_encode")
    return hi, lo


def zorder_decode(hi, lo, n, bits):
    hi = _c(hi, np.uint64)
    lo = _c(lo, np.uint64)
    out = np.zeros((hi.shape[0], n), np.uint32)
    _check(lib().hco_zorder_decode(hi, lo, hi.shape[0], n, bits, out), "zorder_decode")
    return out


def key_int(hi, lo):
    """Python int of a (hi, lo) pair."""
    return (int(hi) << 64) | int(lo)


# ---------------------------------------------------------------------------
# Index
# ---------------------------------------------------------------------------

CURVES = {"hilbert": 0, "zorder": 1}


class Params:
    """Curves, dims per curve, the dimension assignment of Alg. 1 and the kind
    of space-filling curve ("hilbert", the paper's, or "zorder")."""

    def __init__(self, dim=128, curves=8, dpc=16, perm=None, curve="hilbert"):
        self.dim, self.curves, self.dpc, self.bits = dim, curves, dpc, 8
        if perm is None:
            perm = np.arange(curves * dpc)
        self.perm = _c(perm, np.uint16)
        self.curve = CURVES[curve]


def keys(rows, p: Params):
    """Keys of every row and curve: (hi, lo) arrays of shape (rows, curves)."""
    r = _c(rows, np.uint8)
    R = r.shape[0]
    hi = np.zeros((R, p.curves), np.uint64)
    lo = np.zeros((R, p.curves), np.uint64)
    _check(lib().hco_keys_ex(r, R, p.dim, p.perm, p.curves, p.dpc, p.bits, p.curve, hi, lo),
           "keys")
    return hi, lo


class Index:
    """Alg. 1: one list of <key, id> per curve, sorted by (key, id)."""

    def __init__(self, db, p: Params = None):
        self.p = p or Params(dim=db.shape[1])
        self.db = _c(db, np.uint8)
        self.n = self.db.shape[0]
        C = self.p.curves
        self.hi = np.zeros((C, self.n), np.uint64)
        self.lo = np.zeros((C, self.n), np.uint64)
        self.ids = np.zeros((C, self.n), np.uint32)
        _check(lib().hco_build_ex(self.db, self.n, self.p.dim, self.p.perm, C, self.p.dpc,
                                  self.p.bits, self.p.curve, self.hi, self.lo, self.ids),
               "build")

    def _args(self):
        p = self.p
        return (self.hi, self.lo, self.ids)

    def _w(self, w, nq):
        return np.broadcast_to(np.asarray(w, np.uint32), (nq,)).copy()

    def positions(self, queries):
        q = _c(queries, np.uint8)
        p = self.p
        out = np.zeros((q.shape[0], p.curves), np.int64)
        _check(lib().hco_positions(self.hi, self.lo, self.n, p.dim, p.perm, p.curves, p.dpc,
                                   p.bits, p.curve, q, q.shape[0], out), "positions")
        return out

    def candidates(self, queries, w):
        """List of sorted unique candidate-id arrays, one per query."""
        q = _c(queries, np.uint8)
        p = self.p
        nq = q.shape[0]
        wv = self._w(w, nq)
        stride = int(2 * int(wv.max(initial=1)) * p.curves)
        counts = np.zeros(nq, np.uint32)
        ids = np.zeros((nq, max(stride, 1)), np.uint32)
        _check(lib().hco_candidates(self.hi, self.lo, self.ids, self.n, p.dim, p.perm,
                                    p.curves, p.dpc, p.bits, p.curve, q, nq, wv, counts, ids,
                                    max(stride, 1)), "candidates")
        return [ids[i, :counts[i]].copy() for i in range(nq)]

    def search(self, queries, k, w):
        """Alg. 2: (ids, dists) of shape (nq, k), ordered by (dist, id)."""
        q = _c(queries, np.uint8)
        p = self.p
        nq = q.shape[0]
        wv = self._w(w, nq)
        ids = np.zeros((nq, k), np.uint32)
        d = np.zeros((nq, k), np.uint32)
        _check(lib().hco_search(self.hi, self.lo, self.ids, self.db, self.n, p.dim, p.perm,
                                p.curves, p.dpc, p.bits, p.curve, q, nq, k, wv, ids, d),
               "search")
        return ids, d

    def labels(self, queries, k, truth_ids):
        q = _c(queries, np.uint8)
        p = self.p
        out = np.zeros(q.shape[0], np.uint32)
        _check(lib().hco_labels(self.hi, self.lo, self.ids, self.n, p.dim, p.perm, p.curves,
                                p.dpc, p.bits, p.curve, q, q.shape[0], k,
                                _c(truth_ids, np.uint32),
                                out), "labels")
        return out

    def features(self, queries, k):
        q = _c(queries, np.uint8)
        p = self.p
        nq = q.shape[0]
        kv = np.broadcast_to(np.asarray(k, np.uint32), (nq,)).copy()
        out = np.zeros((nq, 24), np.float64)
        _check(lib().hco_features(self.hi, self.lo, self.ids, self.db, self.n, p.dim, p.perm,
                                  p.curves, p.dpc, p.bits, p.curve, q, nq, kv, out),
               "features")
        return out


def lower_bound(hi, lo, qhi, qlo):
    hi = _c(hi, np.uint64)
    lo = _c(lo, np.uint64)
    return int(lib().hco_lower_bound(hi, lo, hi.shape[0], int(qhi), int(qlo)))


def brute_force(db, queries, k):
    """Eq. (3) with ties broken by id: (ids, dists) of shape (nq, k)."""
    db = _c(db, np.uint8)
    q = _c(queries, np.uint8)
    nq = q.shape[0]
    ids = np.zeros((nq, k), np.uint32)
    d = np.zeros((nq, k), np.uint32)
    _check(lib().hco_brute_force(db, db.shape[0], db.shape[1], q, nq, k, ids, d),
           "brute_force")
    return ids, d


# ---------------------------------------------------------------------------
# MLP of the learned probe depth (FP64)
# ---------------------------------------------------------------------------

MLP_DIMS = (24, 64, 64)


def mlp_nparams(dims=MLP_DIMS):
    return int(lib().hco_mlp_nparams(*dims))


def mlp_forward(params, x, dims=MLP_DIMS):
    x = _c(x, np.float64)
    y = np.zeros(x.shape[0], np.float64)
    _check(lib().hco_mlp_forward(_c(params, np.float64), x, x.shape[0], *dims, y),
           "mlp_forward")
    return y


def mlp_loss_grad(params, x, y, dims=MLP_DIMS):
    x = _c(x, np.float64)
    g = np.zeros(mlp_nparams(dims), np.float64)
    loss = ct.c_double(0.0)
    _check(lib().hco_mlp_loss_grad(_c(params, np.float64), x, _c(y, np.float64), x.shape[0],
                                   *dims, g, ct.byref(loss)), "mlp_loss_grad")
    return loss.value, g


def adam_step(theta, m, v, g, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """In-place Adam update of float64 arrays theta, m, v."""
    for a in (theta, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    _check(lib().hco_adam_step(theta, m, v, _c(g, np.float64), theta.shape[0], t, lr, beta1,
                               beta2, eps), "adam_step")
