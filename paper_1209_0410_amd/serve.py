"""Continuous-batching request loop over a resident index (one GPU).

Requests (a query vector and its k) arrive over time.  The loop admits every
request that has arrived into the next batch whenever an in-flight slot is
free and the batch's device memory fits the HBM budget; each batch runs on its
own HIP stream (copy in, per-query w, the uneven search, copy out), so batches
overlap on the device while new requests keep arriving.  This is the online
setting of the paper's Sec. 6 (tasks arrive continuously; the group size is
decided at run time), with slots on streams in place of its CPU/GPU buffers.

With host cores given (a HostSearch and cpu_workers), the loop is the
paper's cooperative scheduler (Sec. 6, Alg. 3): while the requests waiting
are no more than the host workers, each goes to a host core, where one
request costs no device launch; when more are waiting, they are batched for
the GPU as a stream slot frees up, and idle host workers take requests from
the front meanwhile.  Host and GPU give the same rows for a request (same w,
same k), so results do not depend on where a request ran.

The arrival process is seeded: Poisson with a rate that varies sinusoidally,
drawn by thinning (Lewis & Shedler).
"""
import argparse
import collections
import json
import math
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import torch

from . import capi, learned


def sinusoidal_arrivals(duration_s, lo_qps, hi_qps, period_s, seed):
    """Arrival times (s) of a Poisson process with rate
    mid - amp * cos(2 pi t / period), mid = (hi + lo) / 2, amp = (hi - lo) / 2."""
    rng = np.random.default_rng(seed)
    mid, amp = 0.5 * (hi_qps + lo_qps), 0.5 * (hi_qps - lo_qps)
    lam_max = hi_qps
    n = rng.poisson(lam_max * duration_s)
    t = np.sort(rng.uniform(0.0, duration_s, size=n))
    rate = mid - amp * np.cos(2 * math.pi * t / period_s)
    keep = rng.uniform(0.0, lam_max, size=n) < rate
    return t[keep]


def _align(nbytes):
    return (int(nbytes) + 255) & ~255


class HbmBudget:
    """The device memory of the batches in flight (admission control): one
    buffer of `budget` bytes, allocated once when a Server binds it, from which
    each batch takes a block at admission (its inputs, outputs, features, w
    and search scratch) and returns it when the batch is done.  With
    budget_bytes None the budget is the device's free memory less
    reserve_bytes, read before the buffer exists; the Server caps it at what
    its slots can use at once."""

    def __init__(self, budget_bytes=None, reserve_bytes=2 << 30):
        if budget_bytes is None:
            free, _ = torch.cuda.mem_get_info()
            budget_bytes = max(0, free - reserve_bytes)
        self.budget = int(budget_bytes) & ~255
        self.used = 0
        self.peak = 0
        self.refused = 0
        self.buf = None
        self._free = []             # free blocks (offset, bytes), by offset

    def bind(self, device, cap_bytes):
        """Allocates the buffer, of the budget or cap_bytes if that is less."""
        if self.buf is None:
            self.budget = min(self.budget, _align(cap_bytes))
            self.buf = _device_bytes(self.budget, device)
            self._free = [(0, self.budget)] if self.budget else []
        return self

    def largest(self):
        """Bytes of the largest free block."""
        return max((b for _, b in self._free), default=0)

    def take(self, nbytes):
        """Offset of a block of nbytes (the first free one that fits), or None."""
        nbytes = _align(nbytes)
        for i, (o, b) in enumerate(self._free):
            if b >= nbytes:
                if b == nbytes:
                    del self._free[i]
                else:
                    self._free[i] = (o + nbytes, b - nbytes)
                self.used += nbytes
                self.peak = max(self.peak, self.used)
                return o
        return None

    def give(self, off, nbytes):
        """Returns the block taken at off (merged with free neighbours)."""
        nbytes = _align(nbytes)
        self.used -= nbytes
        merged = []
        for o, b in sorted(self._free + [(off, nbytes)]):
            if merged and merged[-1][0] + merged[-1][1] == o:
                merged[-1] = (merged[-1][0], merged[-1][1] + b)
            else:
                merged.append((o, b))
        self._free = merged


def _device_bytes(nbytes, device):
    """A 256-byte-aligned device buffer of nbytes."""
    t = torch.empty(_align(nbytes) + 256, dtype=torch.uint8, device=device)
    off = (-t.data_ptr()) % 256
    return t[off:off + _align(nbytes)]


class _Slot:
    """One stream, its host buffers and, while a batch runs on it, views of
    the batch's device block.  A batch of nq requests travels in one copy each
    way: in, the rows, k and the model's k' packed as [nq x 128 | nq | nq]
    (136 B per request); out, the ids then the distances, nq x k_stride each."""
    IN_BYTES = 136

    def __init__(self, cap, k_stride, dev):
        self.stream = torch.cuda.Stream(device=dev)
        self.k_stride = k_stride
        self.h_in = torch.empty(cap * self.IN_BYTES, dtype=torch.uint8).pin_memory()
        self.h_out = torch.empty(2 * cap * k_stride, dtype=torch.int32).pin_memory()
        self.classes = None          # batch route: (k, first, count) per class
        self.perm = None             # batch route: packed position -> request
        self.done = torch.cuda.Event()
        self.busy = False

    def bind(self, buf, off, layout, nq):
        """Views of a batch's buffers in the block of buf at off."""
        def part(name, dtype):
            o, nb = layout[name]
            return buf[off + o:off + o + nb].view(dtype)
        self.d_in = part("d_in", torch.uint8)
        self.d_out = part("d_out", torch.int32)
        self.scratch = part("scratch", torch.uint8)
        if "w" in layout:
            self.w = part("w", torch.int32)
            self.feat = part("feat", torch.float32).view(nq, learned.FEATURES)
            self.fscratch = part("fscratch", torch.uint8)

    def inputs(self, nq):
        """Device views (rows, k, k') of a batch of nq in d_in."""
        b = self.d_in[:nq * self.IN_BYTES]
        q = b[:nq * 128].view(nq, 128)
        k = b[nq * 128:nq * 132].view(torch.int32)
        kf = b[nq * 132:nq * 136].view(torch.int32)
        return q, k, kf

    def outputs(self, nq, host=False):
        """(ids, dists) of a batch of nq, each nq x k_stride, in d_out or h_out."""
        b = (self.h_out if host else self.d_out)[:2 * nq * self.k_stride]
        m = nq * self.k_stride
        return b[:m].view(nq, self.k_stride), b[m:].view(nq, self.k_stride)


class Server:
    """Admits arriving requests into batches on `slots` streams; with `host`
    (an index.HostSearch) and cpu_workers > 0, short queues go to host cores
    (fixed w only: the learned w is inferred on the GPU).

    route "uneven": one persistent launch per batch with per-request w and k
    (hc_search_uneven; the gather kernel).  route "batch": the batch is packed
    by k on the host and each k class is one hc_search_batch on the automatic
    path, which bands large batches at large w (the row store attached; two
    passes for k > 16) and gathers small ones.  A batch is formed when a slot
    is free and at least min_batch requests wait, or the oldest has waited
    max_wait_s, or no more will arrive."""

    def __init__(self, ix, model=None, w_fixed=64, k_stride=100, max_batch=4096, slots=3,
                 budget=None, cfg=None, w_fallback=None, host=None, cpu_workers=0,
                 k_feature=10, route="uneven", min_batch=1, max_wait_s=0.0, band_min=0):
        if route not in ("uneven", "batch"):
            raise ValueError(f"unknown route {route!r}")
        if route == "batch" and host is not None:
            raise ValueError("the cooperative scheduler uses the uneven route")
        if host is not None and model is not None:
            raise ValueError("the host path takes the fixed w; use model=None with host")
        self.ix = ix
        self.model = model
        self.k_feature = int(k_feature)     # the model's features use min(k, k_feature)
        self.host = host
        self.cpu_workers = int(cpu_workers) if host is not None else 0
        self.w_fixed = int(w_fixed)
        self.w_fallback = int(w_fallback if w_fallback is not None else w_fixed)
        self.k_stride = int(k_stride)
        self.max_batch = int(max_batch)
        self.cfg = cfg
        self.route = route
        self.min_batch = max(1, int(min_batch))
        # batch route: a k class of at least band_min requests takes the banded
        # path whenever each list entry lies in several of its windows, even
        # below the block count the automatic choice wants (0: automatic)
        self.band_min = int(band_min)
        self.max_wait_s = float(max_wait_s)
        dev = ix.db.device
        self._layouts = {}
        self.slots = [_Slot(self.max_batch, self.k_stride, dev) for _ in range(slots)]
        self.budget = budget if budget is not None else HbmBudget()
        self.budget.bind(dev, slots * self.batch_bytes(self.max_batch))

    def _launch(self, slot, hq, hk, hkf, lo, hi):
        if self.route == "batch":
            return self._launch_batch(slot, hq, hk, hkf, lo, hi)
        nq = hi - lo
        # pack the batch on the host (rows, k, k'), then one copy in
        hin = slot.h_in[:nq * _Slot.IN_BYTES].numpy()
        hin[:nq * 128] = hq[lo:hi].reshape(-1)
        hin[nq * 128:nq * 132] = hk[lo:hi].view(np.uint8)
        hin[nq * 132:nq * 136] = hkf[lo:hi].view(np.uint8)
        with torch.cuda.stream(slot.stream):
            slot.d_in[:nq * _Slot.IN_BYTES].copy_(slot.h_in[:nq * _Slot.IN_BYTES],
                                                   non_blocking=True)
            q, k, kf = slot.inputs(nq)
            ids, dists = slot.outputs(nq)
            if self.model is not None:
                kmax = int(self.k_stride)
                capi.call("hc_features", self.ix.handle, ctp(q), nq, kmax, ctp(kf),
                          ctp(slot.feat), ctp(slot.fscratch), slot.fscratch.numel(),
                          stream_of(slot.stream))
                capi.call("hc_mlp_infer", ctp(self.model.bf16), ctp(self.model.norm),
                          ctp(slot.feat), nq, float(self.model.delta), self.model.w_min,
                          self.model.w_max, self.w_fallback, ctp(slot.w), None,
                          stream_of(slot.stream))
                wp = slot.w[:nq]
            else:
                wp = None
            capi.call("hc_search_uneven", self.ix.handle, ctp(q), nq, self.w_fixed,
                      ctp(wp) if wp is not None else None, 1, ctp(k), self.k_stride,
                      ctp(ids), ctp(dists), ctp(slot.scratch), slot.scratch.numel(),
                      _cfgp(self.cfg), stream_of(slot.stream))
            m = 2 * nq * self.k_stride
            slot.h_out[:m].copy_(slot.d_out[:m], non_blocking=True)
            slot.done.record(slot.stream)
        slot.busy = True

    def _layout(self, nq):
        """(name -> (offset, bytes), total) of a batch's device block: the
        input, the outputs, the search scratch and, with a model, the w, the
        features and their scratch; every part 256-byte aligned."""
        if nq not in self._layouts:
            if self.route == "uneven":
                sb = self.ix.uneven_scratch_bytes(nq, self.k_stride, self.cfg)
            else:
                # one search per k class on the automatic path: the scratch of
                # either path for k up to k_stride (banded two passes for k > 16)
                sb = self.ix.scratch_bytes(nq, self.k_stride)
            parts = [("d_in", nq * _Slot.IN_BYTES), ("d_out", 8 * nq * self.k_stride),
                     ("scratch", sb)]
            if self.model is not None:
                parts += [("w", 4 * nq), ("feat", 4 * nq * learned.FEATURES),
                          ("fscratch", self.ix.scratch_bytes(nq))]
            lay, off = {}, 0
            for name, nb in parts:
                lay[name] = (off, nb)
                off += _align(nb)
            self._layouts[nq] = (lay, off)
        return self._layouts[nq]

    def batch_bytes(self, nq):
        """Device bytes a batch of nq requests takes from the budget."""
        return self._layout(nq)[1]

    def _fit(self, avail, want):
        """The largest batch (at most want requests) whose block fits avail bytes."""
        lo, hi = 0, int(want)
        while lo < hi:
            mid = (lo + hi + 1) // 2
            if self.batch_bytes(mid) <= avail:
                lo = mid
            else:
                hi = mid - 1
        return lo

    def _launch_batch(self, slot, hq, hk, hkf, lo, hi):
        """The batch route: requests packed by k (stable), one copy in, the
        learned w for all (if a model is given), one search per k class into
        compact [count x k] blocks (all ids, then all distances), one copy out.
        The host unpacks the blocks (_unpack)."""
        nq = hi - lo
        perm = np.argsort(hk[lo:hi], kind="stable")
        kp = hk[lo:hi][perm]
        classes, o = [], 0
        for kv in np.unique(kp):
            m = int(np.count_nonzero(kp == kv))
            classes.append((int(kv), o, m))
            o += m
        hin = slot.h_in[:nq * _Slot.IN_BYTES].numpy()
        hin[:nq * 128] = hq[lo:hi][perm].reshape(-1)
        hin[nq * 128:nq * 132] = kp.view(np.uint8)
        hin[nq * 132:nq * 136] = hkf[lo:hi][perm].view(np.uint8)
        tot = sum(kv * m for kv, _, m in classes)
        st = stream_of(slot.stream)
        with torch.cuda.stream(slot.stream):
            slot.d_in[:nq * _Slot.IN_BYTES].copy_(slot.h_in[:nq * _Slot.IN_BYTES],
                                                   non_blocking=True)
            q, _, kf = slot.inputs(nq)
            if self.model is not None:
                capi.call("hc_features", self.ix.handle, ctp(q), nq, int(self.k_stride),
                          ctp(kf), ctp(slot.feat), ctp(slot.fscratch), slot.fscratch.numel(),
                          st)
                capi.call("hc_mlp_infer", ctp(self.model.bf16), ctp(self.model.norm),
                          ctp(slot.feat), nq, float(self.model.delta), self.model.w_min,
                          self.model.w_max, self.w_fallback, ctp(slot.w), None, st)
            off = 0
            for kv, first, m in classes:
                qc = q[first:first + m]
                ids = slot.d_out[off:off + m * kv]
                dists = slot.d_out[tot + off:tot + off + m * kv]
                # with a w per request, w_fixed is the typical w (sizes the work)
                wp = ctp(slot.w[first:first + m]) if self.model is not None else None
                wf = self.model.w_hint if self.model is not None else self.w_fixed
                path = capi.HC_PATH_AUTO
                if (self.band_min and m >= self.band_min and kv <= capi.HC_BAND_K_MAX
                        and 2.0 * wf * m >= 3.5 * self.ix.n):
                    path = capi.HC_PATH_BAND
                capi.call("hc_encode_queries", self.ix.handle, ctp(qc), m, ctp(slot.scratch),
                          slot.scratch.numel(), st)
                capi.call("hc_search_encoded_ex", self.ix.handle, ctp(qc), m, kv, int(wf), wp,
                          ctp(ids), ctp(dists), ctp(slot.scratch), slot.scratch.numel(),
                          path, st)
                off += m * kv
            slot.h_out[:2 * tot].copy_(slot.d_out[:2 * tot], non_blocking=True)
            slot.done.record(slot.stream)
        slot.classes, slot.perm, slot.tot = classes, perm, tot
        slot.busy = True

    def _unpack(self, slot, lo, hi, res_ids, res_d):
        """Rows lo..hi-1 of the results from a finished batch-route slot: each
        request's k results, then 0xFFFFFFFF up to k_stride."""
        h = slot.h_out[:2 * slot.tot].numpy().view(np.uint32)
        off = 0
        for kv, first, m in slot.classes:
            rows = lo + slot.perm[first:first + m]
            res_ids[rows] = 0xFFFFFFFF
            res_d[rows] = 0xFFFFFFFF
            res_ids[rows, :kv] = h[off:off + m * kv].reshape(m, kv)
            res_d[rows, :kv] = h[slot.tot + off:slot.tot + off + m * kv].reshape(m, kv)
            off += m * kv

    def run(self, arrivals, queries, ks, keep_results=True, realtime=True, log=None):
        """Serves requests i (arrival time arrivals[i] s, row queries[i], k ks[i]).
        Returns per-request latency (s) and, if asked, the results."""
        R = len(arrivals)
        hq = np.ascontiguousarray(queries, np.uint8)
        hk = np.ascontiguousarray(ks, np.uint32)
        # the model sees k' = min(k, k_feature): the depth it was trained for
        hkf = np.minimum(hk, self.k_feature).astype(np.uint32)
        done_at = np.zeros(R)
        res_ids = np.zeros((R, self.k_stride), np.uint32) if keep_results else None
        res_d = np.zeros((R, self.k_stride), np.uint32) if keep_results else None
        inflight = collections.deque()      # (slot, lo, hi, block offset, bytes)
        cpu_inflight = []                    # futures of host-core requests
        pool = ThreadPoolExecutor(self.cpu_workers) if self.cpu_workers else None
        nxt = 0
        batches = 0
        on_cpu = 0
        sizes = []
        t0 = time.perf_counter()
        clock = (lambda: time.perf_counter() - t0) if realtime else None
        arrivals = np.asarray(arrivals, np.float64)
        next_log = 5.0
        qa = np.ascontiguousarray(queries, np.uint8)
        ka = np.ascontiguousarray(ks, np.uint32)

        def on_host(i):
            ids, d = self.host.search(qa[i:i + 1], w=self.w_fixed, k_stride=self.k_stride,
                                      k_per_query=ka[i:i + 1])
            return i, time.perf_counter() - t0, ids[0], d[0]

        while nxt < R or inflight or cpu_inflight:
            now = clock() if realtime else math.inf
            # retire finished host-core requests
            if cpu_inflight:
                still = []
                for f in cpu_inflight:
                    if f.done():
                        i, t_done, ids, d = f.result()
                        done_at[i] = t_done if realtime else 0.0
                        if keep_results:
                            res_ids[i], res_d[i] = ids, d
                    else:
                        still.append(f)
                cpu_inflight = still
            # retire finished batches (oldest first; each slot records one event)
            for _ in range(len(inflight)):
                slot, lo, hi, boff, nb = inflight[0]
                if not slot.done.query():
                    inflight.rotate(-1)
                    continue
                inflight.popleft()
                t_done = clock() if realtime else 0.0
                done_at[lo:hi] = t_done
                if keep_results and self.route == "batch":
                    self._unpack(slot, lo, hi, res_ids, res_d)
                elif keep_results:
                    hids, hd = slot.outputs(hi - lo, host=True)
                    res_ids[lo:hi] = hids.numpy().view(np.uint32)
                    res_d[lo:hi] = hd.numpy().view(np.uint32)
                slot.busy = False
                self.budget.give(boff, nb)
            if log is not None and realtime and now >= next_log:
                log(f"t={now:.1f}s: {nxt} of {R} admitted, {len(inflight)} batches in flight")
                next_log += 5.0
            # admit what has arrived into a free slot, as much as the budget allows
            arrived = R if not realtime else int(np.searchsorted(arrivals, now, side="right"))
            free = [s for s in self.slots if not s.busy]
            if pool is not None and arrived > nxt:
                idle_cpu = self.cpu_workers - len(cpu_inflight)
                ready = arrived - nxt
                # few waiting: the host cores take them; many waiting and the
                # GPU busy: idle host cores take some from the front
                take = min(ready, idle_cpu) if (ready <= self.cpu_workers or not free) else 0
                for i in range(nxt, nxt + take):
                    cpu_inflight.append(pool.submit(on_host, i))
                nxt += take
                on_cpu += take
            ready_end = min(arrived, nxt + self.max_batch)
            # hold a small batch back while more requests are due soon
            if (realtime and ready_end > nxt and ready_end - nxt < self.min_batch
                    and arrived < R and now - arrivals[nxt] < self.max_wait_s):
                ready_end = nxt
            if ready_end > nxt and free:
                fit = self._fit(self.budget.largest(), ready_end - nxt)
                if fit < 1 and not inflight:
                    raise RuntimeError("HBM budget is below one request's device memory")
                if fit >= 1:
                    end = nxt + fit
                    lay, nb = self._layout(fit)
                    boff = self.budget.take(nb)
                    free[0].bind(self.budget.buf, boff, lay, fit)
                    self._launch(free[0], hq, hk, hkf, nxt, end)
                    inflight.append((free[0], nxt, end, boff, nb))
                    sizes.append(end - nxt)
                    batches += 1
                    nxt = end
                    continue
                self.budget.refused += 1
            if not realtime and not free and inflight:
                inflight[0][0].done.synchronize()
            elif realtime and nxt < R and ready_end == nxt and not inflight and not cpu_inflight:
                time.sleep(max(0.0, min(arrivals[nxt] - now, 0.001)))
            elif cpu_inflight and ready_end == nxt:
                time.sleep(2e-5)            # let the host workers run
        torch.cuda.synchronize()
        if pool is not None:
            pool.shutdown()
        lat = done_at - np.asarray(arrivals) if realtime else None
        stats = {"requests": R, "batches": batches, "on_host_cores": on_cpu,
                 "mean_batch": float(np.mean(sizes)) if sizes else 0.0,
                 "max_batch": int(max(sizes)) if sizes else 0,
                 "hbm_budget": self.budget.budget, "hbm_peak": self.budget.peak,
                 "admission_waits": self.budget.refused}
        if realtime:
            stats.update({"p50_ms": float(np.percentile(lat, 50) * 1e3),
                          "p99_ms": float(np.percentile(lat, 99) * 1e3),
                          "mean_ms": float(lat.mean() * 1e3),
                          "span_s": float(done_at.max()),
                          "sustained_qps": R / float(done_at.max())})
        return stats, (res_ids, res_d)


def ctp(t):
    import ctypes as ct
    return ct.c_void_p(t.data_ptr())


def stream_of(s):
    import ctypes as ct
    return ct.c_void_p(s.cuda_stream)


def _cfgp(cfg):
    import ctypes as ct
    return ct.byref(cfg) if cfg is not None else None


def main(argv=None):
    """The serving scenario: a resident index over n rows, requests arriving at
    a rate that moves sinusoidally between lo and hi per second, k drawn from
    {1, 10, 100}, w per request from the learned model (fixed w as its
    fallback).  Prints one JSON line: latency p50/p99, sustained queries/s,
    batching, and recall@min(k, 10) of the learned and the fixed w on a sample
    of the requests (each searched again alone: results do not depend on the
    mix)."""
    from . import datagen
    from .index import Index, brute_force
    ap = argparse.ArgumentParser(prog="python -m paper_1209_0410_amd.serve")
    ap.add_argument("--n", type=int, default=100_000_000)
    ap.add_argument("--duration", type=float, default=60.0)
    ap.add_argument("--lo", type=float, default=1_000.0)
    ap.add_argument("--hi", type=float, default=200_000.0)
    ap.add_argument("--period", type=float, default=60.0)
    ap.add_argument("--w", type=int, default=16, help="fixed w (the fallback)")
    ap.add_argument("--w-max", type=int, default=64, help="largest learned w")
    ap.add_argument("--train", type=int, default=100_000)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--slots", type=int, default=3)
    ap.add_argument("--max-batch", type=int, default=16_384)
    ap.add_argument("--recall-sample", type=int, default=2_000)
    ap.add_argument("--recall", type=float, default=0.0,
                    help="serve at this recall@10: calibrate the fixed w to it and take "
                         "the batch route with the row store attached (0 = the "
                         "equal-cost comparison of learned and fixed w)")
    ap.add_argument("--min-batch", type=int, default=1)
    ap.add_argument("--max-wait", type=float, default=0.0, help="seconds")
    ap.add_argument("--alone-sample", type=int, default=200,
                    help="served requests searched again alone (recall-target scenario)")
    ap.add_argument("--band-min", type=int, default=0,
                    help="batch route: band a k class of at least this many requests")
    a = ap.parse_args(argv)
    if a.recall > 0:
        return recall_main(a)

    def log(msg):
        print(f"[serve] {msg}", file=sys.stderr, flush=True)

    dev = torch.device("cuda:0")
    t0 = time.time()
    db = datagen.make_db(a.n)
    gdb = torch.from_numpy(db).to(dev)
    del db
    ix = Index(gdb)
    torch.cuda.synchronize()
    log(f"{a.n} rows resident, index {ix.index_bytes / 1e9:.1f} GB, {time.time() - t0:.1f}s")

    # learned w: labels from exact kNN, the model trained on the GPU for the
    # request mix (a request's k, capped at 10: recall is judged on its first
    # 10 results); delta is set so that the mean learned w over the mix equals
    # the fixed w (equal search cost)
    t0 = time.time()
    kmix = np.array([1, 10, 100], np.uint32)
    rng = np.random.default_rng(datagen.SEED_TRAIN)
    rank = learned.ranks(ix)
    tq = torch.from_numpy(datagen.make_queries(a.train, seed=datagen.SEED_TRAIN)).to(dev)
    feats, lab = learned.mixed_k_examples(ix, rank, gdb, tq,
                                          np.minimum(rng.choice(kmix, a.train), 10))
    model = learned.WModel(dev, seed=0, w_min=8, w_max=a.w_max)
    model.set_norm(feats)
    model.train(feats, model.targets(lab), epochs=a.epochs, batch=4096, lr=1e-3, seed=1)
    cq = torch.from_numpy(datagen.make_queries(10_000, seed=datagen.SEED_CALIB)).to(dev)
    ck = np.minimum(rng.choice(kmix, 10_000), 10).astype(np.uint32)
    cf = learned.features(ix, cq, 0, torch.from_numpy(ck.view(np.int32)).to(dev))
    lo_d, hi_d = -16.0, 16.0
    for _ in range(40):
        mid = 0.5 * (lo_d + hi_d)
        if model.windows(cf, mid, a.w).float().mean().item() > a.w:
            hi_d = mid
        else:
            lo_d = mid
    model.delta = lo_d
    del rank, tq, lab, feats
    torch.cuda.synchronize()
    log(f"model trained on {a.train} queries, delta {model.delta:.3f}, {time.time() - t0:.1f}s")

    arrivals = sinusoidal_arrivals(a.duration, a.lo, a.hi, a.period, seed=datagen.SEED_ARRIVALS)
    R = len(arrivals)
    queries = datagen.make_queries(R, seed=datagen.SEED_EVAL)
    ks = np.random.default_rng(datagen.SEED_ARRIVALS).choice(
        np.array([1, 10, 100], np.uint32), size=R)
    log(f"{R} requests over {a.duration:.0f}s, rate {a.lo:.0f} .. {a.hi:.0f} per s")
    srv = Server(ix, model=model, w_fixed=a.w, k_stride=100, max_batch=a.max_batch,
                 slots=a.slots)
    stats, _ = srv.run(arrivals, queries, ks, keep_results=False, realtime=True, log=log)
    log(f"p50 {stats['p50_ms']:.2f} ms, p99 {stats['p99_ms']:.2f} ms, sustained "
        f"{stats['sustained_qps']:.0f} q/s, mean batch {stats['mean_batch']:.0f}")

    # recall on a sample, each request searched alone (same w, same k)
    S = min(a.recall_sample, R)
    sq, sk = queries[:S], ks[:S]
    gsq = torch.from_numpy(sq).to(dev)
    sf = learned.features(ix, gsq, 0, torch.from_numpy(
        np.minimum(sk, 10).astype(np.uint32).view(np.int32)).to(dev))
    mean_w = float(model.windows(sf, None, a.w).float().mean().item())
    rec = {}
    for name, m in (("learned", model), ("fixed", None)):
        s2 = Server(ix, model=m, w_fixed=a.w, k_stride=100, max_batch=1024, slots=1)
        _, (ids, _) = s2.run(np.zeros(S), sq, sk, keep_results=True, realtime=False)
        hits = []
        for k in (1, 10):
            sel = np.nonzero(np.minimum(sk, 10) == k)[0]
            truth, _ = brute_force(gdb, gsq[torch.from_numpy(sel).to(dev)].contiguous(), k)
            truth = truth.cpu().numpy().view(np.uint32)
            hits += [len(set(ids[i, :k].tolist()) & set(truth[j].tolist())) / k
                     for j, i in enumerate(sel)]
        rec[name] = float(np.mean(hits))
    out = {"scenario": "serving loop", "n": a.n, "requests": R, "duration_s": a.duration,
           "rate_qps": [a.lo, a.hi], "period_s": a.period, "k_mix": [1, 10, 100],
           "w_fixed": a.w, "w_max": a.w_max, "delta": model.delta,
           "mean_learned_w_sample": mean_w,
           "recall_at_min_k_10": rec, "recall_sample": S, **stats}
    print(json.dumps(out), flush=True)


def recall_main(a):
    """The serving scenario at a recall target: the fixed w calibrated to
    recall@10 >= target (plus a margin for sampling error) on 10^4
    calibration queries, the row store attached, the batch route (large k
    classes banded, small ones gathered).  Reports latency p50/p99, sustained
    queries/s, the HBM held, recall@min(k, 10) of a sample of the served
    requests, and that each of them equals its result searched alone."""
    from . import datagen
    from .index import Index, brute_force

    def log(msg):
        print(f"[serve] {msg}", file=sys.stderr, flush=True)

    dev = torch.device("cuda:0")
    t0 = time.time()
    db = datagen.make_db(a.n)
    gdb = torch.from_numpy(db).to(dev)
    del db
    ix = Index(gdb)
    rs = ix.attach_rowstore()
    torch.cuda.synchronize()
    log(f"{a.n} rows resident: database {a.n * 128 / 1e9:.1f} GB, index "
        f"{ix.index_bytes / 1e9:.1f} GB, row store {rs / 1e9:.1f} GB, {time.time() - t0:.1f}s")
    cq = torch.from_numpy(datagen.make_queries(10_000, seed=datagen.SEED_CALIB)).to(dev)
    ctruth, _ = brute_force(gdb, cq, 10)
    t0 = time.time()
    w, rc = learned.calibrate_fixed_w(ix, cq, ctruth, 10, a.recall + 0.005, hi=1 << 21)
    del cq, ctruth
    log(f"fixed w = {w} (calibration recall@10 {rc:.4f}) in {time.time() - t0:.1f}s")

    arrivals = sinusoidal_arrivals(a.duration, a.lo, a.hi, a.period, seed=datagen.SEED_ARRIVALS)
    R = len(arrivals)
    queries = datagen.make_queries(R, seed=datagen.SEED_EVAL)
    ks = np.random.default_rng(datagen.SEED_ARRIVALS).choice(
        np.array([1, 10, 100], np.uint32), size=R)
    log(f"{R} requests over {a.duration:.0f}s, rate {a.lo:.0f} .. {a.hi:.0f} per s")
    srv = Server(ix, w_fixed=w, k_stride=100, max_batch=a.max_batch, slots=a.slots,
                 route="batch", min_batch=a.min_batch, max_wait_s=a.max_wait,
                 band_min=a.band_min)
    held = torch.cuda.memory_allocated()
    stats, (ids, d) = srv.run(arrivals, queries, ks, keep_results=True, realtime=True, log=log)
    log(f"p50 {stats['p50_ms']:.2f} ms, p99 {stats['p99_ms']:.2f} ms, sustained "
        f"{stats['sustained_qps']:.0f} q/s, mean batch {stats['mean_batch']:.0f}")
    log("stats " + json.dumps(stats))

    # a sample of the served requests: recall@min(k, 10) against exact kNN; and
    # a smaller sample searched again alone (one request per search, on the
    # uneven path, which splits a wide window over many wavefronts), whose
    # rows must equal the served ones
    S = min(a.recall_sample, R)
    pick = np.linspace(0, R - 1, S).astype(np.int64)
    hits = []
    for kk in (1, 10, 100):
        sel = pick[ks[pick] == kk]
        if not len(sel):
            continue
        kt = min(int(kk), 10)
        truth, _ = brute_force(gdb, torch.from_numpy(queries[sel]).to(dev), kt)
        truth = truth.cpu().numpy().view(np.uint32)
        hits += [len(set(ids[i, :kt].tolist()) & set(truth[j].tolist())) / kt
                 for j, i in enumerate(sel)]
    log(f"recall@min(k, 10) {np.mean(hits):.4f} on {S} served requests")
    alone = pick[::max(1, S // a.alone_sample)]
    same = 0
    for n_done, i in enumerate(alone):
        ai, ad = ix.search_uneven(torch.from_numpy(queries[i:i + 1]).to(dev), w=w,
                                  k=int(ks[i]), k_stride=100)
        same += int((ai.cpu().numpy().view(np.uint32)[0] == ids[i]).all() and
                    (ad.cpu().numpy().view(np.uint32)[0] == d[i]).all())
        if n_done % 50 == 49:
            log(f"searched alone: {n_done + 1} of {len(alone)}, {same} equal")
    out = {"scenario": "serving loop at a recall target", "n": a.n, "requests": R,
           "duration_s": a.duration, "rate_qps": [a.lo, a.hi], "period_s": a.period,
           "k_mix": [1, 10, 100], "w_fixed": w, "calib_recall": rc, "route": "batch",
           "min_batch": a.min_batch, "max_wait_s": a.max_wait, "band_min": a.band_min,
           "recall_at_min_k_10": float(np.mean(hits)), "recall_sample": S,
           "alone_sample": int(len(alone)), "equal_alone": same, "hbm_held_bytes": held,
           "rowstore_bytes": rs, **stats}
    print(json.dumps(out), flush=True)


def cooperative_main(argv=None):
    """The cooperative scheduler against the GPU alone: constant Poisson rates
    over a resident index, fixed w, k from {1, 10, 100}; p50/p99 per rate with
    and without host cores.  Prints one JSON line."""
    from . import datagen
    from .index import HostSearch, Index
    ap = argparse.ArgumentParser(prog="python -m paper_1209_0410_amd.serve --cooperative")
    ap.add_argument("--cooperative", action="store_true")
    ap.add_argument("--n", type=int, default=10_000_000)
    ap.add_argument("--w", type=int, default=16)
    ap.add_argument("--rates", default="1000,5000,20000,100000")
    ap.add_argument("--duration", type=float, default=10.0)
    ap.add_argument("--cpu-workers", type=int, default=12)
    ap.add_argument("--slots", type=int, default=3)
    a = ap.parse_args(argv)

    def log(msg):
        print(f"[serve] {msg}", file=sys.stderr, flush=True)

    dev = torch.device("cuda:0")
    db = datagen.make_db(a.n)
    ix = Index(torch.from_numpy(db).to(dev))
    host = HostSearch(ix, db)
    log(f"{a.n} rows resident on the GPU and in host memory")
    rows = []
    for rate in [float(x) for x in a.rates.split(",")]:
        arr = sinusoidal_arrivals(a.duration, rate, rate, a.duration, seed=datagen.SEED_ARRIVALS)
        R = len(arr)
        q = datagen.make_queries(R, seed=datagen.SEED_EVAL)
        ks = np.random.default_rng(datagen.SEED_ARRIVALS).choice(
            np.array([1, 10, 100], np.uint32), size=R)
        row = {"rate_qps": rate, "requests": R}
        for name, cw in (("gpu", 0), ("cooperative", a.cpu_workers)):
            srv = Server(ix, w_fixed=a.w, k_stride=100, max_batch=16_384, slots=a.slots,
                         host=host if cw else None, cpu_workers=cw)
            st, _ = srv.run(arr, q, ks, keep_results=False, realtime=True)
            row[name] = {k: st[k] for k in ("p50_ms", "p99_ms", "mean_ms", "sustained_qps",
                                            "batches", "mean_batch", "on_host_cores")}
            log(f"rate {rate:.0f}/s {name}: p50 {st['p50_ms']:.3f} ms, p99 "
                f"{st['p99_ms']:.3f} ms, {st['on_host_cores']} of {R} on host cores")
        rows.append(row)
    print(json.dumps({"scenario": "cooperative scheduler", "n": a.n, "w": a.w,
                      "cpu_workers": a.cpu_workers, "duration_s": a.duration,
                      "k_mix": [1, 10, 100], "rates": rows}), flush=True)


if __name__ == "__main__":
    if "--cooperative" in sys.argv[1:]:
        cooperative_main()
    else:
        main()
