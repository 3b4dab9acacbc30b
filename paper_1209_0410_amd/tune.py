"""In-house autotuner of the uneven search's launch shape, and HIP-graph capture.

The tuner times candidate shapes (work-item size in window slots, items per
query, resident wavefronts per CU) of hc_search_uneven on a sample of the
actual batch with HIP events, keeps the fastest, and caches it by workload
signature (database size, batch size, the spread of w and k).
"""
import json
import math
import os

import numpy as np
import torch

from . import capi

CHUNKS = (2048, 4096, 8192, 16384, 32768)
SPLITS = (8, 32)
PER_CU = (0, 8, 12, 16)


def signature(ix, w, k):
    wv = w.float()
    return (f"n{ix.n}|nq{int(math.log2(max(w.numel(), 1)))}|wlog{round(math.log2(wv.mean().item() + 1))}"
            f"|wspread{round((wv.max() / wv.mean().clamp_min(1)).log2().item())}|kmax{int(k.max().item())}")


class Tuner:
    def __init__(self, cache_path=None):
        self.cache_path = cache_path
        self.cache = {}
        if cache_path and os.path.exists(cache_path):
            with open(cache_path) as f:
                self.cache = json.load(f)

    def _time(self, ix, q, w, k, k_stride, cfg, reps=3):
        sc = ix.uneven_scratch(q.shape[0], k_stride, cfg)
        out = (torch.empty((q.shape[0], k_stride), dtype=torch.int32, device=q.device),
               torch.empty((q.shape[0], k_stride), dtype=torch.int32, device=q.device))
        ix.search_uneven(q, w_per_query=w, k_per_query=k, k_stride=k_stride, cfg=cfg, out=out,
                         scratch=sc)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            ix.search_uneven(q, w_per_query=w, k_per_query=k, k_stride=k_stride, cfg=cfg,
                             out=out, scratch=sc)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    def best(self, ix, queries, w, k, sample=20000, log=None):
        """The fastest hc_uneven_cfg for this workload (timed on a sample)."""
        key = signature(ix, w, k)
        if key in self.cache:
            c = self.cache[key]["cfg"]
            return capi.hc_uneven_cfg(*c), self.cache[key]
        m = min(sample, queries.shape[0])
        q, ws, ks = queries[:m].contiguous(), w[:m].contiguous(), k[:m].contiguous()
        k_stride = int(k.max().item())
        results = []
        for ch in CHUNKS:
            for sp in SPLITS:
                for pc in PER_CU:
                    cfg = capi.hc_uneven_cfg(ch, sp, pc)
                    ms = self._time(ix, q, ws, ks, k_stride, cfg)
                    results.append((ms, (ch, sp, pc)))
                    if log:
                        log(f"tune chunk={ch} split={sp} per_cu={pc}: {ms:.3f} ms")
        results.sort()
        ms, c = results[0]
        default_ms = [r for r in results if r[1] == (8192, 32, 0)][0][0]
        entry = {"cfg": list(c), "ms": ms, "default_ms": default_ms, "sample": m,
                 "tried": len(results)}
        self.cache[key] = entry
        if self.cache_path:
            with open(self.cache_path, "w") as f:
                json.dump(self.cache, f, indent=1)
        return capi.hc_uneven_cfg(*c), entry


class Graph:
    """A captured sequence of library calls on fixed buffers, replayed with one
    launch.  Inputs are refreshed by copying into the captured tensors."""

    def __init__(self, fn, warmup=1):
        self.fn = fn
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            for _ in range(warmup):
                fn()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        self.g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.g):
            fn()
        torch.cuda.synchronize()

    def replay(self):
        self.g.replay()
