"""Benchmark of the batched Multicurves search on one MI355X.

Workload: N = 10,000,000 mixture vectors (128 x uint8, 1.28 GB) indexed by 8
curves of 16 dims; a batch of Q = 100,000 queries resident in HBM; k = 10.

One step = one pass of the search path over the batch, through the C ABI:
  fixed w:   hc_encode_queries + hc_search_encoded
  learned w: hc_features (which also encodes the query keys) + hc_mlp_infer +
             hc_search_encoded with the per-query w.
The metric is queries/s at mean recall@10 >= 0.90 (exact kNN truth for the
first --recall-q queries).  Both the fixed w and the learned model's offset
delta are calibrated to that recall on separate calibration queries (seed 5);
the learned model is trained on the GPU on --train queries (seed 3) with
labels from exact kNN.  Also measured: the windows w in --sweep (w = 16, 64,
256 are the plain-method points), each with its recall and the search
kernel's algorithmic HBM bytes / time; p50/p99 of 1,000-query sub-batches;
and the CPU oracle on a bounded sample.

Prints one JSON line on stdout; progress goes to stderr.
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
# MI355X dense int8 matrix-core peak (the banded path's distances are int8
# MFMA products)
MFMA_I8_PEAK_TOPS = 5000.0
TARGET = 0.90
CALIB_TARGET = 0.905    # margin for the sampling error of the evaluation recall


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=10_000_000)
    ap.add_argument("--nq", type=int, default=100_000)
    ap.add_argument("--k", type=int, default=10)
    ap.add_argument("--sweep", default="16,64,256,1024,4096")
    ap.add_argument("--sweep-steps", type=int, default=3)
    ap.add_argument("--recall-q", type=int, default=10_000)
    ap.add_argument("--calib-q", type=int, default=10_000)
    ap.add_argument("--train", type=int, default=200_000, help="0 = no learned w")
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--w-max", type=int, default=1 << 17)
    ap.add_argument("--latency-batch", type=int, default=1000)
    ap.add_argument("--cpu-baseline", type=int, default=1)
    ap.add_argument("--rowstore", type=int, default=1,
                    help="attach the row store (curve-ordered rows) for the banded path")
    ap.add_argument("--f4", type=int, default=1,
                    help="Z-order comparison and incremental insertion (0 = skip)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--w-fixed", type=int, default=0,
                    help="use this fixed w instead of calibrating it (profiling runs)")
    ap.add_argument("--uneven", type=int, default=200_000,
                    help="queries of the uneven batch (per-query w and k); 0 = skip")
    ap.add_argument("--path", default="auto", choices=["auto", "gather", "band"],
                    help="search path of the fixed-w legs (auto: the library's choice)")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="also copy 1 GiB device-to-device 3 times (counter calibration)")
    return ap.parse_args()


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {a.gpus} is not supported "
              "(the multi-GPU design is described, not built)", flush=True)
        sys.exit(2)
    import torch
    from paper_1209_0410_amd import datagen, learned
    from paper_1209_0410_amd.index import Index, brute_force

    dev = torch.device("cuda:0")
    k = a.k
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
    rank = learned.ranks(ix)
    log(f"index build {build_s:.3f}s ({ix.index_bytes / 1e9:.2f} GB)")
    rowstore_bytes, rowstore_s = 0, 0.0
    if a.rowstore:
        t0 = time.time()
        rowstore_bytes = ix.attach_rowstore()
        torch.cuda.synchronize()
        rowstore_s = time.time() - t0
        log(f"row store {rowstore_bytes / 1e9:.2f} GB in {rowstore_s:.3f}s")

    stream = torch.cuda.current_stream()
    sc = ix.scratch(a.nq)
    out = (torch.empty((a.nq, k), dtype=torch.int32, device=dev),
           torch.empty((a.nq, k), dtype=torch.int32, device=dev))

    # exact kNN truth for the first recall-q queries of the batch
    rq = min(a.recall_q, a.nq)
    tid, _ = brute_force(gdb, gq[:rq].contiguous(), k)
    truth = tid.cpu().numpy().view(np.uint32)
    cross = check_truth(db, q, truth, k) if a.cpu_baseline else None
    log(f"truth for {rq} queries" + ("" if cross is None else f"; oracle agrees on {cross}"))

    def recall_of(ids_t):
        return learned.recall_at_k(ids_t[:rq].cpu().numpy().view(np.uint32), truth)

    tstat = {}

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        marks = []
        t_wall = time.perf_counter()
        for _ in range(steps):
            # step start, search start, step end; the search's main kernel
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
            fn(ev, stream)
            marks.append(ev)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t_wall) / steps
        step = [e[0].elapsed_time(e[2]) for e in marks]
        kern = [e[1].elapsed_time(e[2]) for e in marks]
        main = [e[3].elapsed_time(e[4]) for e in marks] \
            if getattr(fn, "main_kernel_events", False) else None
        tstat["main_ms"] = float(np.mean(main)) if main else None
        return float(np.median(step)), float(np.mean(kern)), wall * 1e3

    forced = {"auto": 0, "gather": 1, "band": 2}[a.path]

    def path_of(w):
        return path_name(forced if forced else ix.path(a.nq, k, w, sc.numel()))

    def fixed_step(w):
        def fn(ev=None, st=None):
            if ev: ev[0].record(st)
            ix.encode_queries(gq, sc)
            if ev:
                ev[1].record(st)
                ev[3].record(st)          # creates the events; the search records them again
                ev[4].record(st)
                ix.set_kernel_events(ev[3], ev[4])
            ix.search_encoded(gq, k, w, out, sc, path=forced)
            if ev:
                ix.set_kernel_events()
                ev[2].record(st)
        fn.main_kernel_events = True
        return fn

    def alg_bytes(wsum_slots, union):
        # window ids read + distinct rows gathered + results written
        return 4 * wsum_slots + 128 * union + 8 * k * a.nq

    def window_slots(w_arr):
        pos = ix.positions(gq).cpu().numpy().view(np.uint32).astype(np.int64)
        w_arr = np.broadcast_to(np.asarray(w_arr, np.int64).reshape(-1, 1), pos.shape)
        return int((np.minimum(pos + w_arr, a.n) - np.maximum(pos - w_arr, 0)).sum())

    # ---- fixed-w sweep ---------------------------------------------------------
    rows = []
    if a.copy_probe:
        src = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("copy probe: 3 x 1 GiB device-to-device")

    for w in sorted({int(x) for x in a.sweep.split(",") if x}):
        step_ms, kern_ms, wall_ms = timed(fixed_step(w), a.sweep_steps, 1)
        rec = recall_of(out[0])
        uni = int(learned.union_sizes(ix, rank, gq, w).cpu().numpy().view(np.uint32).sum())
        slots = window_slots(w)
        ab = alg_bytes(slots, uni)
        rows.append(dict(w=w, step_ms=step_ms, kernel_ms=kern_ms, qps=a.nq / step_ms * 1e3,
                         path=path_of(w),
                         recall=rec, union_per_query=uni / a.nq, alg_bytes=ab,
                         alg_GBs=ab / (kern_ms * 1e-3) / 1e9,
                         frac=ab / (kern_ms * 1e-3) / 1e9 / HBM_PEAK_GBS))
        r = rows[-1]
        log(f"fixed w={w} ({r['path']}): {step_ms:.3f} ms/step, {r['qps']:.3e} q/s, "
            f"recall {rec:.4f}, union/q {r['union_per_query']:.0f}, {r['alg_GBs']:.0f} GB/s "
            f"({r['frac']:.1%})")

    # ---- calibration at recall >= 0.90 ------------------------------------------
    cq = datagen.make_queries(a.calib_q, seed=datagen.SEED_CALIB)
    gcq = torch.from_numpy(cq).to(dev)
    ctruth, _ = brute_force(gdb, gcq, k)
    if a.w_fixed:
        w_fix = a.w_fixed
        log(f"fixed w = {w_fix} (given)")
    else:
        w_fix, rec_c = learned.calibrate_fixed_w(ix, gcq, ctruth, k, CALIB_TARGET, hi=a.w_max)
        log(f"calibrated fixed w = {w_fix} (calibration recall {rec_c:.4f})")
    fs, fk, fwall = timed(fixed_step(w_fix), a.steps, a.warmup)
    f_main = tstat["main_ms"]
    f_rec = recall_of(out[0])
    f_out = (out[0].cpu().numpy().view(np.uint32), out[1].cpu().numpy().view(np.uint32))
    f_uni = int(learned.union_sizes(ix, rank, gq, w_fix).cpu().numpy().view(np.uint32).sum())
    f_ab = alg_bytes(window_slots(w_fix), f_uni)
    fixed = dict(w=w_fix, step_ms=fs, kernel_ms=fk, wall_ms=fwall, qps=a.nq / fs * 1e3,
                 recall=f_rec, union_per_query=f_uni / a.nq, alg_bytes=f_ab,
                 alg_GBs=f_ab / (fk * 1e-3) / 1e9, path=path_of(w_fix),
                 alg_TOPs=2 * 128 * f_uni / (fk * 1e-3) / 1e12,
                 alg_ops=2 * 128 * f_uni, main_kernel_ms=f_main)
    log(f"fixed w={w_fix}: {fs:.3f} ms/step, {fixed['qps']:.3e} q/s, recall {f_rec:.4f}; "
        f"search call {fk:.3f} ms, its main kernel {f_main:.3f} ms")

    learned_row = None
    if a.train > 0:
        learned_row = run_learned(a, ix, rank, gdb, gq, gcq, ctruth, out, sc, timed, recall_of,
                                  alg_bytes, window_slots, dev)

    # headline: the faster method whose evaluation recall meets the target
    eligible = [r for r in (fixed, learned_row) if r is not None and r["recall"] >= TARGET]
    head = max(eligible, key=lambda r: r["qps"]) if eligible else fixed
    use_learned = head is learned_row

    # ---- batch latency of the headline method ------------------------------------
    lb = min(a.latency_batch, a.nq)
    lat = []
    for i in range(0, a.nq - lb + 1, lb) if lb > 0 else []:
        sub = gq[i:i + lb]
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        if use_learned:
            learned.search_learned(ix, head["_model"], sub, k,
                                   (out[0][i:i + lb], out[1][i:i + lb]), sc)
        else:
            ix.search(sub, k, w_fix, out=(out[0][i:i + lb], out[1][i:i + lb]), scratch=sc)
        e1.record(stream)
        lat.append((e0, e1))
    torch.cuda.synchronize()
    lat_ms = np.array([e0.elapsed_time(e1) for e0, e1 in lat] or [float("nan")])
    if learned_row is not None:
        learned_row.pop("_model", None)

    uneven = run_uneven(a, ix, rank, gdb, dev) if a.uneven else None
    f4 = run_f4(a, ix, gdb, gq, gcq, ctruth, out, timed, recall_of, w_fix, build_s,
                dev) if a.f4 else None

    cpu = None
    if a.cpu_baseline:
        cpu = cpu_baseline(db, q, k, w_fix, a.cpu_seconds, f_out)

    result = {
        "metric": "queries/s at recall@10≥0.90, learned-w vs fixed-w, 1 GPU; p50/p99 latency",
        "value": head["qps"],
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
        "config": {"workload": f"Multicurves search on one GPU: N={a.n} mixture uint8 d=128, "
                               f"8 curves x 16 dims, Q={a.nq} per batch, k={k}, "
                               f"{'learned' if use_learned else 'fixed'} w calibrated to "
                               f"recall@10>=0.90",
                   "n": a.n, "nq": a.nq, "k": k, "curves": 8,
                   "method": "learned-w" if use_learned else "fixed-w",
                   "rowstore_bytes": rowstore_bytes},
        "recall_at_10": head["recall"],
        "recall_target_met": bool(head["recall"] >= TARGET),
        "recall_queries": rq,
        "fixed_w": fixed,
        "learned_w": learned_row,
        "learned_vs_fixed_qps": (learned_row["qps"] / fixed["qps"]) if learned_row else None,
        "latency_ms": {"batch": lb, "p50": float(np.percentile(lat_ms, 50)),
                       "p99": float(np.percentile(lat_ms, 99))},
        "build_s": build_s,
        "rowstore_s": rowstore_s,
        "sweep": rows,
        "uneven": uneven,
        "f4": f4,
        "roofline": roofline(head, bool(rowstore_bytes)),
    }
    if head is fixed:
        tb, tsrc = counted_traffic(a.n, a.nq, k, w_fix, head["path"])
        if tb is not None:
            result["roofline"]["traffic"] = tb
            result["roofline"]["traffic_source"] = tsrc
    if cpu is not None:
        result["cpu_baseline"] = cpu
    print(json.dumps(result), flush=True)


def run_learned(a, ix, rank, gdb, gq, gcq, ctruth, out, sc, timed, recall_of, alg_bytes,
                window_slots, dev):
    import torch
    from paper_1209_0410_amd import datagen, learned
    from paper_1209_0410_amd.index import brute_force
    k = a.k
    t0 = time.time()
    tq = datagen.make_queries(a.train, seed=datagen.SEED_TRAIN)
    gtq = torch.from_numpy(tq).to(dev)
    ttruth, _ = brute_force(gdb, gtq, k)
    lab = learned.labels(ix, rank, gtq, ttruth)
    feats = learned.features(ix, gtq, k)
    torch.cuda.synchronize()
    labs = lab.cpu().numpy().view(np.uint32)
    log(f"labels for {a.train} training queries in {time.time() - t0:.1f}s; "
        f"w* p10/50/90 = {np.percentile(labs, [10, 50, 90]).tolist()}")
    model = learned.WModel(dev, seed=0, w_min=8, w_max=a.w_max)
    model.set_norm(feats)
    y = model.targets(lab)
    t0 = time.time()
    losses = model.train(feats, y, epochs=a.epochs, batch=4096, lr=1e-3, seed=1)
    torch.cuda.synchronize()
    train_s = time.time() - t0
    log(f"trained {a.epochs} epochs in {train_s:.1f}s, loss {losses[0]:.3f} -> {losses[-1]:.3f}")
    cfeats = learned.features(ix, gcq, k)
    delta, rec_c = learned.calibrate_delta(ix, model, gcq, cfeats, ctruth, k, CALIB_TARGET)
    model.delta = delta
    log(f"calibrated delta = {delta:.3f} (calibration recall {rec_c:.4f})")
    feats_b = torch.empty((a.nq, learned.FEATURES), dtype=torch.float32, device=dev)
    wq = torch.empty(a.nq, dtype=torch.int32, device=dev)

    def fn(ev=None, st=None):
        if ev is None:
            learned.search_learned(ix, model, gq, k, out, sc, feats=feats_b, w=wq)
            return
        ev[0].record(st)
        _learned_split(ix, model, gq, k, out, sc, feats_b, wq, ev, st)
        ev[2].record(st)

    ls, lk, lwall = timed(fn, a.steps, a.warmup)
    rec = recall_of(out[0])
    wv = wq.cpu().numpy().view(np.uint32)
    uni = int(learned.union_sizes(ix, rank, gq, 0, wq).cpu().numpy().view(np.uint32).sum())
    ab = alg_bytes(window_slots(wv.astype(np.int64)), uni)
    row = dict(step_ms=ls, kernel_ms=lk, wall_ms=lwall, qps=a.nq / ls * 1e3, recall=rec,
               path=path_name(ix.path(a.nq, k, model.w_hint, sc.numel())),
               alg_TOPs=2 * 128 * uni / (lk * 1e-3) / 1e12,
               delta=delta, mean_w=float(wv.mean()),
               w_pct=np.percentile(wv, [10, 50, 90, 99]).tolist(),
               union_per_query=uni / a.nq, alg_bytes=ab, alg_GBs=ab / (lk * 1e-3) / 1e9,
               train_queries=a.train, epochs=a.epochs, loss=[losses[0], losses[-1]],
               train_s=train_s)
    log(f"learned: {ls:.3f} ms/step, {row['qps']:.3e} q/s, recall {rec:.4f}, mean w "
        f"{row['mean_w']:.0f}")
    row["_model"] = model
    return row


def path_name(p):
    return {1: "gather", 2: "band"}[p]


def roofline(head, rowstore):
    """Roofline of the search's main kernel, timed with HIP events that the
    library records on its stream around that kernel alone (else, for a step
    without them, around the whole hc_search_encoded call): HBM-bound on the
    gather path (window ids + distinct rows + results per call); on the banded
    path the distances are int8 matrix-core products, 2 x 128 ops per distinct
    candidate per call, against the dense int8 MFMA peak.  With the row store
    attached the banded kernel is k_band_dma (tiles copied into LDS), else
    k_band (rows gathered by id)."""
    km = head.get("main_kernel_ms")
    alone = km is not None
    km = km if alone else head["kernel_ms"]
    if head["path"] == "gather":
        ach = head["alg_bytes"] / (km * 1e-3) / 1e9
        return {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": ach / HBM_PEAK_GBS, "traffic": None,
                "kernel": "k_stream" + ("" if alone else " (the whole gather call)"),
                "kernel_ms": km, "call_ms": head["kernel_ms"],
                "alg_bytes_per_launch": head["alg_bytes"]}
    ops = head.get("alg_ops", head["alg_TOPs"] * 1e12 * head["kernel_ms"] * 1e-3)
    ach = ops / (km * 1e-3) / 1e12
    return {"bound": "mfma", "achieved": ach, "peak": MFMA_I8_PEAK_TOPS,
            "unit": "TOP/s", "frac": ach / MFMA_I8_PEAK_TOPS, "traffic": None,
            "kernel": ("k_band_dma" if rowstore else "k_band")
                      + ("" if alone else " with k_band_place/k_scan_excl/k_band_scatter/"
                         "k_band_merge (the whole banded call)"),
            "kernel_ms": km, "call_ms": head["kernel_ms"], "alg_ops_per_launch": ops}


KERNEL_SOURCES = {"gather": ("k_stream", ("hc_search.hip", "hc_device.h")),
                  "band": ("k_band_dma", ("hc_band.hip", "hc_search.hip", "hc_device.h",
                                      "hc_scan.h"))}


def sources_md5(path):
    import hashlib
    src = os.path.join(ROOT, "paper_1209_0410_amd", "csrc")
    return hashlib.md5(b"".join(open(os.path.join(src, f), "rb").read()
                                for f in KERNEL_SOURCES[path][1])).hexdigest()


def counted_traffic(n, nq, k, w, path):
    """HBM bytes per search call from the committed rocprofv3 counter summary of
    this workload, if its kernel sources are the ones built here; else None."""
    import glob
    md5 = sources_md5(path)
    want = f"workload: n={n} nq={nq} k={k} w={w}"
    kern = KERNEL_SOURCES[path][0]
    for path in glob.glob(os.path.join(ROOT, "profiles", f"{kern}_*_counters.md")):
        text = open(path).read()
        if want not in text or f"kernel_sources_md5: {md5}" not in text:
            continue
        for line in text.splitlines():
            if line.startswith("traffic_bytes_per_launch:"):
                return float(line.split(":")[1]), os.path.relpath(path, ROOT)
    return None, None


def run_f4(a, ix, gdb, gq, gcq, ctruth, out, timed, recall_of, w_fix, build_s, dev):
    """The Z-order curve in place of the Hilbert curve (same data, same
    calibration), and rows appended to a built index without a rebuild."""
    import torch
    from paper_1209_0410_amd import learned
    from paper_1209_0410_amd.index import Index
    k = a.k
    zx = Index(gdb, curve="zorder")
    zsc = zx.scratch(a.nq)
    rec_h_w = None

    def step(w):
        def fn(ev=None, st=None):
            if ev is not None:
                ev[0].record(st)
                ev[1].record(st)
            zx.search(gq, k, w, out=out, scratch=zsc)
            if ev is not None:
                ev[2].record(st)
        return fn

    timed(step(w_fix), 1, 1)
    rec_h_w = recall_of(out[0])
    w_z, rec_c = learned.calibrate_fixed_w(zx, gcq, ctruth, k, CALIB_TARGET, hi=1 << 20)
    zs, zk, _ = timed(step(w_z), a.steps, a.warmup)
    z = dict(recall_at_hilbert_w=rec_h_w, hilbert_w=w_fix, w=w_z, calib_recall=rec_c,
             step_ms=zs, qps=a.nq / zs * 1e3, recall=recall_of(out[0]))
    log(f"z-order: recall {rec_h_w:.4f} at the Hilbert w={w_fix}; needs w={w_z} for "
        f"{CALIB_TARGET}: {zs:.3f} ms/step, {z['qps']:.3e} q/s, recall {z['recall']:.4f}")
    del zx, zsc
    # insertion: the last 1% of the rows appended to an index over the rest
    m = max(1, a.n // 100)
    base = Index(gdb[:a.n - m])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ins = base.insert(gdb)
    torch.cuda.synchronize()
    ins_s = time.perf_counter() - t0
    same = all(torch.equal(ins.curve(c)[0], ix.curve(c)[0]) and
               torch.equal(ins.curve(c)[1], ix.curve(c)[1]) for c in range(8))
    ins_row = dict(n0=a.n - m, m=m, insert_s=ins_s, full_build_s=build_s,
                   equals_full_build=bool(same))
    log(f"insert {m} rows into {a.n - m}: {ins_s:.3f}s (full build {build_s:.3f}s), "
        f"equal to the full build: {same}")
    del base, ins
    return {"zorder": z, "insert": ins_row}


def run_uneven(a, ix, rank, gdb, dev):
    """Uneven batch: w log-uniform in [8, 512] and k from {1, 10, 100} per query,
    one autotuned persistent launch, captured in a HIP graph and replayed."""
    import torch
    from paper_1209_0410_amd import datagen, learned
    from paper_1209_0410_amd.index import brute_force
    from paper_1209_0410_amd.tune import Graph, Tuner
    nq = a.uneven
    q = datagen.make_queries(nq, seed=datagen.SEED_UNEVEN)
    w, k = datagen.uneven_w_k(nq)
    gq = torch.from_numpy(q).to(dev)
    gw = torch.from_numpy(w.view(np.int32)).to(dev)
    gk = torch.from_numpy(k.view(np.int32)).to(dev)
    kst = int(k.max())
    t0 = time.time()
    # shapes timed on the whole batch: a sample's best shape is not the batch's
    cfg, entry = Tuner().best(ix, gq, gw, gk, sample=nq)
    log(f"uneven: tuned {entry['tried']} shapes in {time.time() - t0:.1f}s: "
        f"chunk={cfg.chunk_slots} split={cfg.max_split} per_cu={cfg.blocks_per_cu} "
        f"({entry['ms']:.3f} ms vs default {entry['default_ms']:.3f} ms on {entry['sample']})")
    sc = ix.uneven_scratch(nq, kst, cfg)
    out = (torch.empty((nq, kst), dtype=torch.int32, device=dev),
           torch.empty((nq, kst), dtype=torch.int32, device=dev))
    g = Graph(lambda: ix.search_uneven(gq, w_per_query=gw, k_per_query=gk, k_stride=kst,
                                       cfg=cfg, out=out, scratch=sc))
    for _ in range(a.warmup):
        g.replay()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(a.steps)]
    for e0, e1 in ev:
        e0.record()
        g.replay()
        e1.record()
    torch.cuda.synchronize()
    ms = float(np.median([e0.elapsed_time(e1) for e0, e1 in ev]))
    uni = int(learned.union_sizes(ix, rank, gq, 0, gw).cpu().numpy().view(np.uint32).sum())
    pos = ix.positions(gq).cpu().numpy().view(np.uint32).astype(np.int64)
    wl = w.astype(np.int64)[:, None]
    slots = int((np.minimum(pos + wl, a.n) - np.maximum(pos - wl, 0)).sum())
    ab = 4 * slots + 128 * uni + 8 * int(k.sum())
    # recall@min(k, 10) on the first queries (exact kNN with k = 10)
    m = min(nq, 2000)
    tid, _ = brute_force(gdb, gq[:m].contiguous(), 10)
    truth = tid.cpu().numpy().view(np.uint32)
    got = out[0][:m].cpu().numpy().view(np.uint32)
    hits = [len(set(got[i, :min(int(k[i]), 10)].tolist()) & set(truth[i, :min(int(k[i]), 10)].tolist()))
            / min(int(k[i]), 10) for i in range(m)]
    row = dict(nq=nq, ms_per_batch=ms, qps=nq / ms * 1e3, mean_w=float(w.mean()),
               k_mix={str(v): int((k == v).sum()) for v in np.unique(k)},
               cfg=[cfg.chunk_slots, cfg.max_split, cfg.blocks_per_cu], tune=entry,
               union_per_query=uni / nq, alg_bytes=ab, alg_GBs=ab / (ms * 1e-3) / 1e9,
               recall_at_min_k_10=float(np.mean(hits)), graph=True)
    log(f"uneven: {ms:.3f} ms per batch of {nq}, {row['qps']:.3e} q/s, "
        f"{row['alg_GBs']:.0f} GB/s, recall@min(k,10) {row['recall_at_min_k_10']:.4f}")
    return row


def _learned_split(ix, model, gq, k, out, sc, feats_b, wq, ev, st):
    """The learned step with an event between the MLP and the search kernel."""
    from paper_1209_0410_amd import capi, learned
    from paper_1209_0410_amd.index import _ptr, _stream
    nq = gq.shape[0]
    capi.call("hc_features", ix.handle, _ptr(gq), nq, int(k), None, _ptr(feats_b), _ptr(sc),
              sc.numel(), _stream())
    capi.call("hc_mlp_infer", _ptr(model.bf16), _ptr(model.norm), _ptr(feats_b), nq,
              float(model.delta), model.w_min, model.w_max, 64, _ptr(wq), None, _stream())
    ev[1].record(st)
    ix.search_encoded(gq, k, model.w_hint, out, sc, w_per_query=wq)


def check_truth(db, q, truth, k, m=16):
    """The GPU exact kNN against the oracle's on the first m queries."""
    import oracle
    ids, _ = oracle.brute_force(db, q[:m], k)
    if not (ids == truth[:m]).all():
        raise AssertionError("GPU brute force differs from the oracle")
    return f"{m} queries"


def cpu_baseline(db, q, k, w, seconds, gpu_out):
    """The oracle's search timed on the host cores on a bounded query sample;
    its results must equal the timed GPU step's (gpu_out) on every sampled query."""
    import oracle
    t0 = time.time()
    oix = oracle.Index(db)
    build = time.time() - t0
    log(f"oracle index build {build:.1f}s")
    t0 = time.time()
    probe = 128
    oix.search(q[:probe], k, w)
    per = (time.time() - t0) / probe
    sample = int(min(len(q), max(probe, seconds / max(per, 1e-9))))
    t0 = time.time()
    rid, rd = oix.search(q[:sample], k, w)
    dt = time.time() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    log(f"oracle search {sample} queries in {dt:.1f}s on {threads} threads")
    if not ((gpu_out[0][:sample] == rid).all() and (gpu_out[1][:sample] == rd).all()):
        raise AssertionError("the timed GPU step differs from the oracle on the sample")
    log(f"timed GPU step equals the oracle on all {sample} sampled queries")
    return {"value": sample / dt, "unit": "queries/s", "cores": threads, "kind": "oracle",
            "sample": f"first {sample} queries of the batch at the calibrated fixed w={w}, "
                      f"k={k}, same N; the oracle's own index, built in {build:.1f}s "
                      f"(not timed); its results equal the timed GPU step's on all of them"}


if __name__ == "__main__":
    main()
