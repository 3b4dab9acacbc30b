"""Benchmark of the batched Multicurves search on one MI355X.

One step = one pass of the search path (query keys, binary search, windows,
union, distances, top-k) over a batch of Q queries resident in HBM, through
the C ABI (hc_search_batch = hc_encode_queries + hc_search_encoded).

Workload (default): N = 10,000,000 mixture vectors (128 x uint8, 1.28 GB),
8 curves of 16 dims, Q = 100,000 queries, k = 10, w in {16, 64, 256}.
Prints one JSON line (see the keys below).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=10_000_000)
    ap.add_argument("--nq", type=int, default=100_000)
    ap.add_argument("--k", type=int, default=10)
    ap.add_argument("--w", type=int, default=64, help="w of the headline line")
    ap.add_argument("--sweep", default="16,64,256", help="w values measured")
    ap.add_argument("--recall-q", type=int, default=1000)
    ap.add_argument("--latency-batch", type=int, default=1000)
    ap.add_argument("--cpu-baseline", type=int, default=1)
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="queries of the oracle sample (0 = sized to ~15 s)")
    return ap.parse_args()


def recall_at(ids, truth):
    k = truth.shape[1]
    hits = [len(set(a.tolist()) & set(b.tolist())) for a, b in zip(ids, truth)]
    return float(np.mean(hits)) / k


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {a.gpus} is not supported "
              "(the multi-GPU design is described, not built)", flush=True)
        sys.exit(2)
    import torch
    from paper_1209_0410_amd import datagen
    from paper_1209_0410_amd.index import Index, brute_force

    dev = torch.device("cuda:0")
    t0 = time.time()
    db = datagen.make_db(a.n)
    q = datagen.make_queries(a.nq)
    log(f"data n={a.n} nq={a.nq} in {time.time() - t0:.1f}s")
    gdb = torch.from_numpy(db).to(dev)
    gq = torch.from_numpy(q).to(dev)
    torch.cuda.synchronize()
    t0 = time.time()
    ix = Index(gdb)
    torch.cuda.synchronize()
    build_s = time.time() - t0
    log(f"index build {build_s:.3f}s ({ix.index_bytes / 1e9:.2f} GB)")

    k = a.k
    stream = torch.cuda.current_stream()
    sc = ix.scratch(a.nq)
    out = (torch.empty((a.nq, k), dtype=torch.int32, device=dev),
           torch.empty((a.nq, k), dtype=torch.int32, device=dev))

    # recall truth: exact kNN on the GPU for the first recall-q queries
    rq = min(a.recall_q, a.nq)
    tid, _ = brute_force(gdb, gq[:rq].contiguous(), k)
    truth = tid.cpu().numpy().view(np.uint32)
    log(f"brute-force truth for {rq} queries")

    sweep = sorted({int(x) for x in a.sweep.split(",") if x} | {a.w})
    rows = {}
    for w in sweep:
        for _ in range(a.warmup):
            ix.search(gq, k, w, out=out, scratch=sc)
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
               torch.cuda.Event(enable_timing=True)) for _ in range(a.steps)]
        torch.cuda.synchronize()
        t_wall = time.perf_counter()
        for e0, e1, e2 in ev:
            e0.record(stream)
            ix.encode_queries(gq, sc)
            e1.record(stream)
            ix.search_encoded(gq, k, w, out, sc)
            e2.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t_wall
        step_ms = [e0.elapsed_time(e2) for e0, _, e2 in ev]
        kern_ms = [e1.elapsed_time(e2) for _, e1, e2 in ev]
        enc_ms = [e0.elapsed_time(e1) for e0, e1, _ in ev]
        ids = out[0][:rq].cpu().numpy().view(np.uint32)
        rec = recall_at(ids, truth)
        # algorithmic bytes of the search kernel: window ids, distinct rows, results
        wsum = 0
        ucount = None
        if 16 * w <= 4096:
            counts, _ = ix.candidates(gq, w)
            ucount = counts.cpu().numpy().view(np.uint32).astype(np.int64)
        pos = ix.positions(gq).cpu().numpy().view(np.uint32).astype(np.int64)
        lo = np.maximum(pos - w, 0)
        hi = np.minimum(pos + w, a.n)
        wsum = int((hi - lo).sum())
        rows[w] = dict(w=w, step_ms=float(np.median(step_ms)), kernel_ms=float(np.mean(kern_ms)),
                       kernel_ms_median=float(np.median(kern_ms)),
                       encode_ms=float(np.mean(enc_ms)), wall_ms=wall * 1e3 / a.steps,
                       recall=rec, window_ids=wsum,
                       unique=None if ucount is None else int(ucount.sum()))
        r = rows[w]
        if r["unique"] is not None:
            alg = 4 * wsum + 128 * r["unique"] + 8 * k * a.nq
            r["alg_bytes"] = alg
            r["alg_GBs"] = alg / (r["kernel_ms"] * 1e-3) / 1e9
        log(f"w={w} step {r['step_ms']:.3f} ms kernel {r['kernel_ms']:.3f} ms "
            f"q/s {a.nq / r['step_ms'] * 1e3:.3e} recall@{k} {rec:.4f} "
            f"U/q {None if r['unique'] is None else r['unique'] / a.nq:.1f} "
            f"GB/s {r.get('alg_GBs', 0):.0f}")

    head = rows[a.w]
    # batch latency: sub-batches timed one by one
    lb = min(a.latency_batch, a.nq)
    lat = []
    for i in range(0, a.nq - lb + 1, lb):
        sub = gq[i:i + lb]
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        ix.search(sub, k, a.w, out=(out[0][i:i + lb], out[1][i:i + lb]), scratch=sc)
        e1.record(stream)
        lat.append((e0, e1))
    torch.cuda.synchronize()
    lat_ms = np.array([e0.elapsed_time(e1) for e0, e1 in lat])

    cpu = None
    if a.cpu_baseline:
        cpu = cpu_baseline(db, q, k, a.w, a.cpu_sample)

    result = {
        "metric": "queries/s at recall@10≥0.90, learned-w vs fixed-w, 1 GPU; p50/p99 latency",
        "value": a.nq / (head["step_ms"] * 1e-3),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": head["step_ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": f"plain method on GPU: N={a.n} mixture uint8 d=128, 8 curves x 16 "
                               f"dims, Q={a.nq}, k={k}, fixed w={a.w}",
                   "n": a.n, "nq": a.nq, "k": k, "w": a.w, "curves": 8},
        "recall_at_10": head["recall"],
        "recall_target_met": bool(head["recall"] >= 0.90),
        "recall_queries": rq,
        "latency_ms": {"batch": lb, "p50": float(np.percentile(lat_ms, 50)),
                       "p99": float(np.percentile(lat_ms, 99))},
        "build_s": build_s,
        "sweep": [{kk: v for kk, v in r.items()} for r in rows.values()],
    }
    if head.get("alg_GBs") is not None:
        result["roofline"] = {"bound": "hbm", "achieved": head["alg_GBs"], "peak": HBM_PEAK_GBS,
                              "unit": "GB/s", "frac": head["alg_GBs"] / HBM_PEAK_GBS,
                              "traffic": None, "kernel": "k_search",
                              "kernel_ms": head["kernel_ms"],
                              "alg_bytes_per_launch": head["alg_bytes"]}
    if cpu is not None:
        result["cpu_baseline"] = cpu
    print(json.dumps(result), flush=True)


def cpu_baseline(db, q, k, w, sample):
    """The oracle's search, timed on the host cores on a bounded query sample."""
    import oracle
    t0 = time.time()
    oix = oracle.Index(db)
    build = time.time() - t0
    log(f"oracle index build {build:.1f}s")
    if sample <= 0:
        t0 = time.time()
        oix.search(q[:200], k, w)
        per = (time.time() - t0) / 200
        sample = int(min(len(q), max(200, 15.0 / max(per, 1e-9))))
    t0 = time.time()
    oix.search(q[:sample], k, w)
    dt = time.time() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    log(f"oracle search {sample} queries in {dt:.1f}s on {threads} threads")
    return {"value": sample / dt, "unit": "queries/s", "cores": threads, "kind": "oracle",
            "sample": f"first {sample} of the batch's queries, same index shape and w={w}, "
                      f"k={k}; oracle index built separately in {build:.1f}s"}


if __name__ == "__main__":
    main()
