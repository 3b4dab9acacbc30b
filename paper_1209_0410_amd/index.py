"""Index and search over device tensors, through the C ABI.

PyTorch supplies device memory and the current HIP stream; every step of the
index build and of the search runs in libhypercurves.so.
"""
import ctypes as ct

import numpy as np
import torch

from . import capi


def _ptr(t):
    return ct.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return ct.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check_rows(x, name):
    if not (x.is_cuda and x.dtype == torch.uint8 and x.dim() == 2 and x.shape[1] == 128
            and x.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous (n, 128) uint8 CUDA tensor")
    if x.data_ptr() % 16:
        raise ValueError(f"{name} must be 16-byte aligned")


def _empty_bytes(nbytes, device):
    t = torch.empty(max(int(nbytes), 256) + 256, dtype=torch.uint8, device=device)
    off = (-t.data_ptr()) % 256
    return t[off:off + max(int(nbytes), 256)]


def encode_keys(rows, curves=8, perm=None, curve="hilbert"):
    """Keys (Hilbert, or Z-order) of every row and curve: int64 tensor
    (rows, curves, 2) of {hi, lo}."""
    _check_rows(rows, "rows")
    p, keep = capi.make_params(curves=curves, perm=perm, curve=curve)
    out = torch.empty((rows.shape[0], curves, 2), dtype=torch.int64, device=rows.device)
    capi.call("hc_encode_keys", ct.byref(p), _ptr(rows), rows.shape[0], _ptr(out), _stream())
    del keep
    return out


class Index:
    """Alg. 1 index of a resident uint8 database (n, 128) on one GPU.  `curve`:
    "hilbert" (the method's) or "zorder" (for comparison)."""

    def __init__(self, db, curves=8, perm=None, curve="hilbert"):
        _check_rows(db, "db")
        self.db = db
        self.n = db.shape[0]
        self.curves = curves
        self.curve_kind = curve
        self.perm = None if perm is None else [int(x) for x in perm]
        self._p, self._keep = capi.make_params(curves=curves, perm=self.perm, curve=curve)
        ib, sb = ct.c_size_t(), ct.c_size_t()
        capi.call("hc_index_bytes", ct.byref(self._p), self.n, ct.byref(ib), ct.byref(sb))
        self.index_bytes = ib.value
        self.buf = _empty_bytes(ib.value, db.device)
        scratch = _empty_bytes(sb.value, db.device)
        h = ct.c_void_p()
        capi.call("hc_build_index", ct.byref(self._p), _ptr(db), self.n, _ptr(self.buf),
                  ib.value, _ptr(scratch), sb.value, _stream(), ct.byref(h))
        self.handle = h
        self._scratch = None
        torch.cuda.current_stream().synchronize()
        del scratch

    @classmethod
    def attach(cls, db, buf, curves=8, perm=None, curve="hilbert"):
        """Handle over an index buffer restored from a previous build."""
        self = cls.__new__(cls)
        _check_rows(db, "db")
        self.db, self.n, self.curves = db, db.shape[0], curves
        self.curve_kind = curve
        self.perm = None if perm is None else [int(x) for x in perm]
        self._p, self._keep = capi.make_params(curves=curves, perm=self.perm, curve=curve)
        self.buf = buf
        self.index_bytes = buf.numel()
        h = ct.c_void_p()
        capi.call("hc_index_attach", ct.byref(self._p), _ptr(db), self.n, _ptr(buf),
                  buf.numel(), ct.byref(h))
        self.handle = h
        self._scratch = None
        return self

    def attach_rowstore(self):
        """Builds and attaches the row store (the rows of every curve in list
        order, for the banded path); returns its size in bytes."""
        sz = ct.c_size_t()
        capi.call("hc_rowstore_bytes", self.handle, ct.byref(sz))
        self.rowstore = _empty_bytes(sz.value, self.db.device)
        capi.call("hc_rowstore_build", self.handle, _ptr(self.rowstore), sz.value, _stream())
        return sz.value

    def detach_rowstore(self):
        capi.call("hc_rowstore_detach", self.handle)
        self.rowstore = None

    def insert(self, db):
        """Index over `db`, whose first n rows are this index's rows, made by
        inserting rows n .. (no rebuild); equal to Index(db) bit for bit.  This
        index stays valid."""
        _check_rows(db, "db")
        m = db.shape[0] - self.n
        if m < 1:
            raise ValueError("db must hold more rows than the index")
        ib, sb = ct.c_size_t(), ct.c_size_t()
        capi.call("hc_insert_bytes", self.handle, m, ct.byref(ib), ct.byref(sb))
        new = Index.__new__(Index)
        new.db, new.n, new.curves = db, db.shape[0], self.curves
        new.curve_kind, new.perm = self.curve_kind, self.perm
        new._p, new._keep = capi.make_params(curves=self.curves, perm=self.perm,
                                             curve=self.curve_kind)
        new.index_bytes = ib.value
        new.buf = _empty_bytes(ib.value, db.device)
        scratch = _empty_bytes(sb.value, db.device)
        h = ct.c_void_p()
        capi.call("hc_insert_rows", self.handle, _ptr(db), m, _ptr(new.buf), ib.value,
                  _ptr(scratch), sb.value, _stream(), ct.byref(h))
        new.handle = h
        new._scratch = None
        torch.cuda.current_stream().synchronize()
        del scratch
        return new

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            try:
                capi.load().hc_index_destroy(h)
            except Exception:
                pass
            self.handle = None

    # -- helpers --------------------------------------------------------------
    def scratch_bytes(self, nq, k_max=16):
        """Scratch bytes of a batch of nq queries with k up to k_max on either
        path (hc_search_scratch_bytes_k)."""
        sz = ct.c_size_t()
        capi.call("hc_search_scratch_bytes_k", self.handle, nq, int(k_max), ct.byref(sz))
        return sz.value

    def scratch(self, nq, k_max=16):
        """The index's shared scratch, grown to hold a batch of nq queries with
        k up to k_max on either path."""
        nb = self.scratch_bytes(nq, k_max)
        if self._scratch is None or self._scratch.numel() < nb:
            self._scratch = _empty_bytes(nb, self.db.device)
        return self._scratch

    def path(self, nq, k, w, scratch_bytes=None):
        """Execution path hc_search_encoded takes (capi.HC_PATH_GATHER / _BAND)."""
        if scratch_bytes is None:
            scratch_bytes = self.scratch(nq, k).numel()
        p = ct.c_uint32()
        capi.call("hc_search_choose_path", self.handle, nq, k, int(w), scratch_bytes,
                  ct.byref(p))
        return p.value

    def new_scratch(self, nq, k_max=16):
        """A scratch buffer of its own (for concurrent streams)."""
        return _empty_bytes(self.scratch_bytes(nq, k_max), self.db.device)

    def curve(self, c):
        """(keys int64 (n, 2) of {hi, lo}, ids int32 (n,)) views of curve c's list."""
        kp, ip = ct.c_void_p(), ct.c_void_p()
        capi.call("hc_index_curve", self.handle, c, ct.byref(kp), ct.byref(ip))
        base = self.buf.data_ptr()
        ko = (kp.value - base)
        io = (ip.value - base)
        keys = self.buf[ko:ko + 16 * self.n].view(torch.int64).view(self.n, 2)
        ids = self.buf[io:io + 4 * self.n].view(torch.int32)
        return keys, ids

    # -- search ---------------------------------------------------------------
    def search(self, queries, k, w=64, w_per_query=None, out=None, scratch=None, path=0):
        """Alg. 2: (ids, dists) int32 tensors (nq, k); uint32 values, 0xFFFFFFFF = empty."""
        _check_rows(queries, "queries")
        nq = queries.shape[0]
        if out is None:
            ids = torch.empty((nq, k), dtype=torch.int32, device=queries.device)
            dists = torch.empty((nq, k), dtype=torch.int32, device=queries.device)
        else:
            ids, dists = out
        sc = scratch if scratch is not None else self.scratch(nq, k)
        wp = None
        if w_per_query is not None:
            assert w_per_query.dtype == torch.int32 and w_per_query.is_cuda
            wp = _ptr(w_per_query)
        capi.call("hc_encode_queries", self.handle, _ptr(queries), nq, _ptr(sc), sc.numel(),
                  _stream())
        capi.call("hc_search_encoded_ex", self.handle, _ptr(queries), nq, k, int(w or 0), wp,
                  _ptr(ids), _ptr(dists), _ptr(sc), sc.numel(), int(path), _stream())
        return ids, dists

    def encode_queries(self, queries, scratch):
        """First launch of search(): query keys into `scratch`."""
        capi.call("hc_encode_queries", self.handle, _ptr(queries), queries.shape[0],
                  _ptr(scratch), scratch.numel(), _stream())

    def set_kernel_events(self, begin=None, end=None):
        """torch.cuda.Event pair recorded around the search's main kernel by
        later searches on this index (None, None: off).  Each event must have
        been recorded once, so that it exists."""
        capi.call("hc_index_set_kernel_events", self.handle,
                  begin.cuda_event if begin is not None else None,
                  end.cuda_event if end is not None else None)

    def search_encoded(self, queries, k, w, out, scratch, w_per_query=None, path=0):
        """Second launch of search(): keys already in `scratch`.  path: 0 auto,
        1 gather, 2 banded (capi.HC_PATH_*)."""
        ids, dists = out
        wp = _ptr(w_per_query) if w_per_query is not None else None
        capi.call("hc_search_encoded_ex", self.handle, _ptr(queries), queries.shape[0], k,
                  int(w or 0), wp, _ptr(ids), _ptr(dists), _ptr(scratch), scratch.numel(),
                  int(path), _stream())
        return ids, dists

    def uneven_scratch_bytes(self, nq, k_stride, cfg=None):
        sz = ct.c_size_t()
        capi.call("hc_uneven_scratch_bytes", self.handle, nq, k_stride,
                  ct.byref(cfg) if cfg is not None else None, ct.byref(sz))
        return sz.value

    def uneven_scratch(self, nq, k_stride, cfg=None):
        return _empty_bytes(self.uneven_scratch_bytes(nq, k_stride, cfg), self.db.device)

    def search_uneven(self, queries, w=0, k=10, w_per_query=None, k_per_query=None,
                      k_stride=None, cfg=None, out=None, scratch=None):
        """Per-query w and k in one persistent launch: (ids, dists) int32 (nq, k_stride),
        row q holding k_q results then 0xFFFFFFFF."""
        _check_rows(queries, "queries")
        nq = queries.shape[0]
        if k_stride is None:
            k_stride = int(k_per_query.max().item()) if k_per_query is not None else int(k)
        if out is None:
            out = (torch.empty((nq, k_stride), dtype=torch.int32, device=queries.device),
                   torch.empty((nq, k_stride), dtype=torch.int32, device=queries.device))
        sc = scratch if scratch is not None else self.uneven_scratch(nq, k_stride, cfg)
        capi.call("hc_search_uneven", self.handle, _ptr(queries), nq, int(w),
                  _ptr(w_per_query) if w_per_query is not None else None, int(k),
                  _ptr(k_per_query) if k_per_query is not None else None, k_stride,
                  _ptr(out[0]), _ptr(out[1]), _ptr(sc), sc.numel(),
                  ct.byref(cfg) if cfg is not None else None, _stream())
        return out

    def positions(self, queries):
        _check_rows(queries, "queries")
        nq = queries.shape[0]
        out = torch.empty((nq, self.curves), dtype=torch.int32, device=queries.device)
        sc = self.scratch(nq)
        capi.call("hc_positions", self.handle, _ptr(queries), nq, _ptr(out), _ptr(sc),
                  sc.numel(), _stream())
        return out

    def candidates(self, queries, w=64, w_per_query=None, stride=None):
        """(counts int32 (nq,), ids int32 (nq, stride)); row q holds counts[q] ids, unordered."""
        _check_rows(queries, "queries")
        nq = queries.shape[0]
        if stride is None:
            stride = 16 * int(w)
        counts = torch.empty(nq, dtype=torch.int32, device=queries.device)
        ids = torch.empty((nq, max(stride, 1)), dtype=torch.int32, device=queries.device)
        sc = self.scratch(nq)
        wp = _ptr(w_per_query) if w_per_query is not None else None
        capi.call("hc_candidates", self.handle, _ptr(queries), nq, int(w), wp, _ptr(counts),
                  _ptr(ids), stride, _ptr(sc), sc.numel(), _stream())
        return counts, ids


def brute_force(db, queries, k):
    """Eq. (3) exact kNN on the GPU: (ids, dists) int32 tensors (nq, k)."""
    _check_rows(db, "db")
    _check_rows(queries, "queries")
    nq = queries.shape[0]
    sz = ct.c_size_t()
    capi.call("hc_brute_force_scratch_bytes", db.shape[0], nq, k, ct.byref(sz))
    sc = _empty_bytes(sz.value, db.device)
    ids = torch.empty((nq, k), dtype=torch.int32, device=db.device)
    dists = torch.empty((nq, k), dtype=torch.int32, device=db.device)
    capi.call("hc_brute_force", _ptr(db), db.shape[0], _ptr(queries), nq, k, _ptr(ids),
              _ptr(dists), _ptr(sc), sc.numel(), _stream())
    return ids, dists


class HostSearch:
    """Host copies of an index's curve lists and of its database: the CPU side
    of the cooperative scheduler (the paper's Alg. 3).  search() runs Alg. 2 on
    the calling thread through the same library (ctypes releases the GIL, so
    calls on several threads run in parallel); its rows equal
    Index.search_uneven's bit for bit."""

    def __init__(self, ix, db_host):
        self.ix = ix
        sz = ct.c_size_t()
        capi.call("hc_host_index_bytes", ix.handle, ct.byref(sz))
        self.lists = np.empty(sz.value, np.uint8)
        capi.call("hc_host_index_copy", ix.handle, self.lists.ctypes.data_as(ct.c_void_p),
                  sz.value, _stream())
        self.db = np.ascontiguousarray(db_host, dtype=np.uint8)
        if self.db.shape != (ix.n, 128):
            raise ValueError("db_host must be the index's (n, 128) uint8 database")

    def search(self, queries, w=16, k=10, k_stride=None, w_per_query=None, k_per_query=None,
               out=None):
        """(ids, dists) uint32 arrays (nq, k_stride) for host queries (nq, 128)."""
        q = np.ascontiguousarray(queries, dtype=np.uint8)
        nq = q.shape[0]
        if k_stride is None:
            k_stride = int(np.max(k_per_query)) if k_per_query is not None else int(k)
        if out is None:
            out = (np.empty((nq, k_stride), np.uint32), np.empty((nq, k_stride), np.uint32))

        def p(a):
            return None if a is None else np.ascontiguousarray(a, np.uint32).ctypes.data_as(
                ct.c_void_p)
        wp = None if w_per_query is None else np.ascontiguousarray(w_per_query, np.uint32)
        kp = None if k_per_query is None else np.ascontiguousarray(k_per_query, np.uint32)
        capi.call("hc_host_search", self.ix.handle, self.lists.ctypes.data_as(ct.c_void_p),
                  self.db.ctypes.data_as(ct.c_void_p), q.ctypes.data_as(ct.c_void_p), nq,
                  int(w), p(wp), int(k), p(kp), k_stride,
                  out[0].ctypes.data_as(ct.c_void_p), out[1].ctypes.data_as(ct.c_void_p))
        return out
