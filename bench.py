"""Benchmark of the batched Multicurves search on one MI355X.

Headline workload (the learned-probe-depth configuration): N = 50,000,000
mixture vectors (128 x uint8, 6.4 GB) indexed by 8 curves of 16 dims; the
MLP that predicts each query's w is trained on 1,000,000 queries (seed 3)
labelled from exact kNN; the fixed w and the learned model's offset delta are
both calibrated to recall@10 >= 0.90 on 10,000 queries (seed 5); the timed
batch is 100,000 fresh evaluation queries (seed 4), resident in HBM, k = 10,
and recall@10 is measured on all of them against exact kNN.

One step = one pass of the search path over the batch, through the C ABI:
  fixed w:   hc_encode_queries + hc_search_encoded
  learned w: hc_features (which also encodes the query keys) + hc_mlp_infer +
             hc_search_encoded with the per-query w.
The headline value is the faster of the two whose evaluation recall meets the
target; both are reported, with their ratio.

Secondary legs on the first 10,000,000 rows of the same database (a prefix):
the plain-method windows w = 16, 64, 256 (and wider) with their recall and
roofline, fixed w at recall 0.90, the uneven batch (per-query w and k, one
persistent launch in a HIP graph), the Z-order curve and incremental
insertion.  Also: the streaming-read bandwidth of the device, the timed step
with the query upload and result download, p50/p99 of 1,000-query
sub-batches, and the CPU oracle on a bounded sample of the batch (all host
threads and one), whose results must equal the timed step's.

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
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=50_000_000, help="database rows of the headline")
    ap.add_argument("--nq", type=int, default=100_000, help="evaluation queries (the batch)")
    ap.add_argument("--k", type=int, default=10)
    ap.add_argument("--train", type=int, default=1_000_000, help="0 = no learned w")
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--confidence", type=lambda x: [float(v) for v in x.split(",")],
                    default=[1.0, 0.5, 0.25, 0.0],
                    help="weights of the MLP's prediction against its training mean to try")
    ap.add_argument("--calib-q", type=int, default=10_000)
    ap.add_argument("--w-max", type=int, default=1 << 20)
    ap.add_argument("--w-fixed", type=int, default=0,
                    help="use this fixed w instead of calibrating it (profiling runs)")
    ap.add_argument("--truth-check", type=int, default=256,
                    help="evaluation queries whose GPU exact kNN is checked against the oracle")
    ap.add_argument("--latency-batch", type=int, default=1000)
    ap.add_argument("--rowstore", type=int, default=1,
                    help="attach the row store (curve-ordered rows) for the banded path")
    ap.add_argument("--path", default="auto", choices=["auto", "gather", "band"],
                    help="search path of the timed fixed-w steps (auto: the library's choice)")
    ap.add_argument("--secondary-n", type=int, default=10_000_000,
                    help="rows of the secondary legs (a prefix of the database); 0 = skip them")
    ap.add_argument("--sweep", default="16,64,256,1024,4096")
    ap.add_argument("--sweep-steps", type=int, default=10)
    ap.add_argument("--uneven", type=int, default=200_000,
                    help="queries of the uneven batch (per-query w and k); 0 = skip")
    ap.add_argument("--f4", type=int, default=1,
                    help="Z-order comparison and incremental insertion (0 = skip)")
    ap.add_argument("--cpu-baseline", type=int, default=1)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--cpu-seconds-1t", type=float, default=6.0)
    ap.add_argument("--probe-gib", type=int, default=8,
                    help="GiB read by the streaming-read probe (0 = skip)")
    ap.add_argument("--power-seconds", type=float, default=5.0,
                    help="repeat the headline step this long while sampling power and clock "
                         "(0 = skip)")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="also copy 1 GiB device-to-device 3 times (counter calibration)")
    return ap.parse_args()


# ---------------------------------------------------------------------------
# timing helpers
# ---------------------------------------------------------------------------

def timed(fn, steps, warmup, stream, warm_s=0.0):
    """Runs fn(ev, stream) `steps` times after `warmup` untimed runs, and after
    further untimed runs until warm_s seconds have passed (a short step that
    follows host-only work would otherwise be timed before the clocks rise).
    fn records ev[0] at the step's start, ev[1] before the search call, ev[2]
    at the end; a search step also hands ev[3], ev[4] to the library, which
    records them around the search's main kernel.  Returns per-step lists (ms)."""
    import torch
    t0 = time.perf_counter()
    for _ in range(warmup):
        fn(None, stream)
    torch.cuda.synchronize()
    while time.perf_counter() - t0 < warm_s:
        fn(None, stream)
        torch.cuda.synchronize()
    marks = []
    t_wall = time.perf_counter()
    for _ in range(steps):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
        fn(ev, stream)
        marks.append(ev)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t_wall) / steps * 1e3
    step = [e[0].elapsed_time(e[2]) for e in marks]
    call = [e[1].elapsed_time(e[2]) for e in marks]
    main = [e[3].elapsed_time(e[4]) for e in marks] if getattr(fn, "main_events", False) \
        else None
    return dict(step=step, call=call, main=main, wall_ms=wall)


def summary(t):
    """Median, min and max of each timed quantity."""
    out = {"step_ms": float(np.median(t["step"])), "step_ms_min": float(np.min(t["step"])),
           "step_ms_max": float(np.max(t["step"])), "call_ms": float(np.median(t["call"])),
           "wall_ms": t["wall_ms"]}
    if t["main"]:
        out["main_kernel_ms"] = float(np.mean(t["main"]))
        out["main_kernel_ms_min"] = float(np.min(t["main"]))
        out["main_kernel_ms_max"] = float(np.max(t["main"]))
    return out


def fixed_step(ix, gq, k, w, out, sc, path):
    def fn(ev, st):
        if ev:
            ev[0].record(st)
        ix.encode_queries(gq, sc)
        if ev:
            ev[1].record(st)
            ev[3].record(st)          # creates the events; the search records them again
            ev[4].record(st)
            ix.set_kernel_events(ev[3], ev[4])
        ix.search_encoded(gq, k, w, out, sc, path=path)
        if ev:
            ix.set_kernel_events()
            ev[2].record(st)
    fn.main_events = True
    return fn


def learned_step(ix, model, gq, k, out, sc, feats_b, wq):
    from paper_1209_0410_amd import capi
    from paper_1209_0410_amd.index import _ptr, _stream
    nq = gq.shape[0]

    def fn(ev, st):
        if ev:
            ev[0].record(st)
        capi.call("hc_features", ix.handle, _ptr(gq), nq, int(k), None, _ptr(feats_b), _ptr(sc),
                  sc.numel(), _stream())
        capi.call("hc_mlp_infer", _ptr(model.bf16), _ptr(model.norm), _ptr(feats_b), nq,
                  float(model.delta), model.w_min, model.w_max, 64, _ptr(wq), None, _stream())
        if ev:
            ev[1].record(st)
            ev[3].record(st)
            ev[4].record(st)
            ix.set_kernel_events(ev[3], ev[4])
        ix.search_encoded(gq, k, model.w_hint, out, sc, w_per_query=wq)
        if ev:
            ix.set_kernel_events()
            ev[2].record(st)
    fn.main_events = True
    return fn


def path_name(p):
    return {1: "gather", 2: "band"}[p]


def u32(t):
    return t.cpu().numpy().view(np.uint32)


# ---------------------------------------------------------------------------
# algorithmic work of a search call
# ---------------------------------------------------------------------------

class Work:
    """Algorithmic bytes (gather path) and int8 ops (banded path) of one
    search call over a batch, from the window sizes and the union sizes
    (hc_union_sizes, exact)."""

    def __init__(self, ix, rank, gq, k):
        self.ix, self.rank, self.gq, self.k = ix, rank, gq, k
        self.pos = u32(ix.positions(gq)).astype(np.int64)

    def of(self, w=None, w_per_query=None):
        from paper_1209_0410_amd import learned
        n = self.ix.n
        if w_per_query is not None:
            uni = int(u32(learned.union_sizes(self.ix, self.rank, self.gq, 0,
                                              w_per_query)).astype(np.int64).sum())
            wl = u32(w_per_query).astype(np.int64)[:, None]
        else:
            uni = int(u32(learned.union_sizes(self.ix, self.rank, self.gq,
                                              w)).astype(np.int64).sum())
            wl = np.int64(w)
        slots = int((np.minimum(self.pos + wl, n) - np.maximum(self.pos - wl, 0)).sum())
        nq = self.gq.shape[0]
        # gather: window ids read + distinct rows gathered + results written
        alg_bytes = 4 * slots + 128 * uni + 8 * self.k * nq
        # banded: 128 multiply-adds (2 x 128 ops) per distinct candidate
        alg_ops = 2 * 128 * uni
        return dict(union_per_query=uni / nq, slots_per_query=slots / nq, alg_bytes=alg_bytes,
                    alg_ops=alg_ops)


def roofline_of(path, work, kernel_ms, counted=None):
    """Roofline of one search call's main kernel: HBM-bound on the gather path
    (algorithmic bytes per launch / kernel time vs 8 TB/s); on the banded path
    the rows are shared by the queries of a block and the distances are int8
    matrix-core products, so the figure is algorithmic ops per launch / kernel
    time vs the dense int8 peak (5.0 POP/s), with the counted HBM bytes beside
    it when a counter summary of this workload exists."""
    if path == "gather":
        ach = work["alg_bytes"] / (kernel_ms * 1e-3) / 1e9
        return {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": ach / HBM_PEAK_GBS, "traffic": counted, "kernel": "k_stream",
                "kernel_ms": kernel_ms, "alg_bytes_per_launch": work["alg_bytes"]}
    ach = work["alg_ops"] / (kernel_ms * 1e-3) / 1e12
    return {"bound": "mfma", "achieved": ach, "peak": MFMA_I8_PEAK_TOPS, "unit": "TOP/s",
            "frac": ach / MFMA_I8_PEAK_TOPS, "traffic": counted, "kernel": "k_band_dma",
            "kernel_ms": kernel_ms, "alg_ops_per_launch": work["alg_ops"]}


KERNEL_SOURCES = {"gather": ("k_stream", ("hc_search.hip", "hc_device.h")),
                  "band": ("k_band_dma", ("hc_band.hip", "hc_search.hip", "hc_device.h",
                                      "hc_scan.h"))}


def sources_md5(path):
    import hashlib
    src = os.path.join(ROOT, "paper_1209_0410_amd", "csrc")
    return hashlib.md5(b"".join(open(os.path.join(src, f), "rb").read()
                                for f in KERNEL_SOURCES[path][1])).hexdigest()


def counted_traffic(workload, path):
    """HBM bytes per launch of the main kernel from a committed rocprofv3 counter
    summary of this workload, if its kernel sources are the ones built here."""
    import glob
    md5 = sources_md5(path)
    kern = KERNEL_SOURCES[path][0]
    for f in glob.glob(os.path.join(ROOT, "profiles", f"{kern}_*_counters.md")):
        text = open(f).read()
        if f"workload: {workload}\n" not in text or f"kernel_sources_md5: {md5}" not in text:
            continue
        for line in text.splitlines():
            if line.startswith("traffic_bytes_per_launch:"):
                return float(line.split(":")[1]), os.path.relpath(f, ROOT)
    return None, None


# ---------------------------------------------------------------------------
# main
# ---------------------------------------------------------------------------

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
    stream = torch.cuda.current_stream()
    k = a.k
    nrows = max(a.n, a.secondary_n)
    t0 = time.time()
    db = datagen.make_db(nrows)
    q = datagen.make_queries(a.nq, seed=datagen.SEED_EVAL)
    log(f"data: {nrows} rows, {a.nq} evaluation queries in {time.time() - t0:.1f}s")
    gdb_all = torch.from_numpy(db).to(dev)
    gdb = gdb_all[:a.n]
    gq = torch.from_numpy(q).to(dev)
    torch.cuda.synchronize()
    t0 = time.time()
    ix = Index(gdb)
    torch.cuda.synchronize()
    build_s = time.time() - t0
    rank = learned.ranks(ix)
    log(f"index over {a.n} rows in {build_s:.3f}s ({ix.index_bytes / 1e9:.2f} GB)")
    rowstore_bytes = 0
    if a.rowstore:
        rowstore_bytes = ix.attach_rowstore()
        torch.cuda.synchronize()
        log(f"row store {rowstore_bytes / 1e9:.2f} GB")
    sc = ix.scratch(a.nq, a.k)
    out = (torch.empty((a.nq, k), dtype=torch.int32, device=dev),
           torch.empty((a.nq, k), dtype=torch.int32, device=dev))

    # exact kNN truth for every evaluation query; the oracle checks a sample
    t0 = time.time()
    # recall@10 (of the first min(k, 10) results for k below 10): the exact
    # kNN truth is taken to that depth
    kt = min(k, 10)
    tid, _ = brute_force(gdb, gq, kt)
    truth = u32(tid)
    log(f"exact kNN of {a.nq} evaluation queries in {time.time() - t0:.1f}s")

    def recall_of(ids_t):
        return learned.recall_at_k(u32(ids_t), truth)

    forced = {"auto": 0, "gather": 1, "band": 2}[a.path]
    work = Work(ix, rank, gq, k)

    # ---- fixed w at recall >= 0.90 ----------------------------------------
    cq = datagen.make_queries(a.calib_q, seed=datagen.SEED_CALIB)
    gcq = torch.from_numpy(cq).to(dev)
    ctruth, _ = brute_force(gdb, gcq, kt)
    t0 = time.time()
    if a.w_fixed:
        w_fix, rec_c = a.w_fixed, None
        log(f"fixed w = {w_fix} (given)")
    else:
        w_fix, rec_c = learned.calibrate_fixed_w(ix, gcq, ctruth, k, CALIB_TARGET, hi=a.w_max)
        log(f"calibrated fixed w = {w_fix} (calibration recall {rec_c:.4f}) in "
            f"{time.time() - t0:.1f}s")
    f_path = forced if forced else ix.path(a.nq, k, w_fix, sc.numel())
    ft = summary(timed(fixed_step(ix, gq, k, w_fix, out, sc, forced), a.steps, a.warmup,
                       stream))
    fixed_out = (u32(out[0]), u32(out[1]))
    fw = work.of(w=w_fix)
    fixed = dict(w=w_fix, calib_recall=rec_c, path=path_name(f_path), **ft,
                 qps=a.nq / ft["step_ms"] * 1e3, recall=recall_of(out[0]), **fw)
    log(f"fixed w={w_fix} ({fixed['path']}): {ft['step_ms']:.3f} ms/step "
        f"[{ft['step_ms_min']:.3f}, {ft['step_ms_max']:.3f}], {fixed['qps']:.3e} q/s, "
        f"recall {fixed['recall']:.4f}; main kernel {ft.get('main_kernel_ms', 0):.3f} ms")

    # ---- learned w ----------------------------------------------------------
    learned_row, model, learned_out, wq = None, None, None, None
    if a.train > 0 and k > 16:
        log("learned w skipped: its labels take the exact top-k, k <= 16")
    elif a.train > 0:
        learned_row, model, learned_out, wq = run_learned(a, ix, rank, gdb, gq, gcq, ctruth,
                                                          out, sc, recall_of, work, stream, dev)

    eligible = [r for r in (fixed, learned_row) if r is not None and r["recall"] >= TARGET]
    head = max(eligible, key=lambda r: r["qps"]) if eligible else fixed
    use_learned = head is learned_row
    head_out = learned_out if use_learned else fixed_out

    # ---- the headline step with the query upload and result download --------
    e2e = end_to_end(a, ix, model if use_learned else None, q, k, w_fix, sc, forced, stream,
                     dev)
    log(f"end to end (upload, step, download): {e2e['ms']:.3f} ms, {e2e['qps']:.3e} q/s")

    # ---- batch latency of the headline method -------------------------------
    lat = sub_batch_latency(a, ix, model if use_learned else None, gq, k, w_fix, out, sc,
                            stream)
    log(f"{lat['batch']}-query sub-batches: p50 {lat['p50']:.3f} ms, p99 {lat['p99']:.3f} ms")

    # ---- the device's streaming-read bandwidth ------------------------------
    # ---- power and clock under the headline step ----------------------------
    power = power_leg(a, learned_step(ix, model, gq, k, out, sc,
                                      torch.empty((a.nq, 24), dtype=torch.float32, device=dev),
                                      torch.empty(a.nq, dtype=torch.int32, device=dev))
                      if use_learned else fixed_step(ix, gq, k, w_fix, out, sc, forced),
                      stream)
    if power:
        log(f"power: {power['socket_power_W']:.0f} W, GFX clock {power['gfx_clock_MHz']:.0f} MHz "
            f"over {power['steps']} steps ({power['samples']} samples)")

    probe = read_probe(a, dev) if a.probe_gib else None
    if probe:
        log(f"streaming read: {probe['GBs']:.0f} GB/s ({probe['bytes'] / 2**30:.0f} GiB, "
            f"{probe['runs']} runs)")

    # ---- the GPU truth against the oracle; the oracle's own timing -----------
    cpu, check = None, None
    if a.cpu_baseline:
        check, cpu = oracle_legs(a, db[:a.n], q, truth, kt, k, w_fix, fixed_out, learned_out,
                                 None if wq is None else u32(wq), use_learned, ix, rank, gq,
                                 dev)

    workload = (f"Multicurves search, learned probe depth: N={a.n} mixture uint8 d=128, "
                f"8 curves x 16 dims, Q={a.nq} fresh evaluation queries per batch, k={k}, "
                f"recall@10>=0.90; learned w trained on {a.train} labelled queries")
    wkey = f"n={a.n} nq={a.nq} k={k} " + (f"learned train={a.train}" if use_learned
                                          else f"w={w_fix}")
    hk = "band" if head["path"] == "band" else "gather"
    tb, tsrc = counted_traffic(wkey, hk)
    roof = roofline_of(head["path"], head, head["main_kernel_ms"], tb)
    roof["call_ms"] = head["call_ms"]
    if tsrc:
        roof["traffic_source"] = tsrc

    secondary = run_secondary(a, gdb_all, db, k, dev, stream) if a.secondary_n else None

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
        "config": {"workload": workload, "n": a.n, "nq": a.nq, "k": k, "curves": 8,
                   "train_queries": a.train, "calib_queries": a.calib_q,
                   "method": "learned-w" if use_learned else "fixed-w",
                   "rowstore_bytes": rowstore_bytes},
        "recall_at_10": head["recall"],
        "recall_target_met": bool(head["recall"] >= TARGET),
        "recall_queries": a.nq,
        "fixed_w": fixed,
        "learned_w": learned_row,
        "learned_vs_fixed_qps": (learned_row["qps"] / fixed["qps"]) if learned_row else None,
        "step_ms_min": head["step_ms_min"],
        "step_ms_max": head["step_ms_max"],
        "end_to_end": e2e,
        "latency_ms": lat,
        "read_probe": probe,
        "power": power,
        "build_s": build_s,
        "truth_check": check,
        "secondary": secondary,
        "roofline": roof,
    }
    if cpu is not None:
        result["cpu_baseline"] = cpu
    print(json.dumps(result), flush=True)


def run_learned(a, ix, rank, gdb, gq, gcq, ctruth, out, sc, recall_of, work, stream, dev):
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
    labs = u32(lab)
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
    # a batch of training queries (as many as the evaluation batch) on which
    # the confidence in the prediction is chosen by speed
    gsel = gtq[:a.nq].clone()
    del gtq, ttruth, feats, y
    cfeats = learned.features(ix, gcq, k)
    feats_b = torch.empty((a.nq, learned.FEATURES), dtype=torch.float32, device=dev)
    wq = torch.empty(a.nq, dtype=torch.int32, device=dev)
    # For each confidence lam (prediction y_mean + lam (y - y_mean)): the
    # offset delta that reaches the recall target on the calibration queries,
    # then the step time on the training batch.  The fastest lam is kept.
    t0 = time.time()
    grid = []
    for lam in a.confidence:
        model.set_confidence(lam)
        d, r = learned.calibrate_delta(ix, model, gcq, cfeats, ctruth, k, CALIB_TARGET)
        model.delta = d
        ts = summary(timed(learned_step(ix, model, gsel, k, out, sc, feats_b, wq), 3, 1,
                           stream))
        grid.append(dict(confidence=lam, delta=d, calib_recall=r, w_hint=model.w_hint,
                         train_batch_ms=ts["step_ms"], mean_w=float(u32(wq).mean())))
        log(f"confidence {lam:.2f}: delta {d:.3f} (calibration recall {r:.4f}), mean w "
            f"{grid[-1]['mean_w']:.0f}, {ts['step_ms']:.3f} ms on {a.nq} training queries")
    best = min(grid, key=lambda g: g["train_batch_ms"])
    model.set_confidence(best["confidence"])
    model.delta, model.w_hint = best["delta"], best["w_hint"]
    delta, rec_c = best["delta"], best["calib_recall"]
    del gsel
    log(f"chosen confidence {best['confidence']:.2f}, delta = {delta:.3f} in "
        f"{time.time() - t0:.1f}s")
    lt = summary(timed(learned_step(ix, model, gq, k, out, sc, feats_b, wq), a.steps, a.warmup,
                       stream))
    lout = (u32(out[0]), u32(out[1]))
    wv = u32(wq)
    lw = work.of(w_per_query=wq)
    row = dict(path=path_name(ix.path(a.nq, k, model.w_hint, sc.numel())), **lt,
               qps=a.nq / lt["step_ms"] * 1e3, recall=recall_of(out[0]), delta=delta,
               calib_recall=rec_c, mean_w=float(wv.mean()),
               w_pct=np.percentile(wv, [10, 50, 90, 99]).tolist(), **lw,
               confidence=best["confidence"], confidence_grid=grid,
               train_queries=a.train, epochs=a.epochs, loss=[losses[0], losses[-1]],
               train_s=train_s, label_pct=np.percentile(labs, [10, 50, 90]).tolist())
    log(f"learned: {lt['step_ms']:.3f} ms/step [{lt['step_ms_min']:.3f}, "
        f"{lt['step_ms_max']:.3f}], {row['qps']:.3e} q/s, recall {row['recall']:.4f}, "
        f"mean w {row['mean_w']:.0f}; main kernel {lt.get('main_kernel_ms', 0):.3f} ms")
    return row, model, lout, wq


def end_to_end(a, ix, model, q, k, w_fix, sc, forced, stream, dev):
    """The headline step with the batch uploaded from pinned host memory before
    it and the results downloaded after it, all on the stream: median of the
    timed runs."""
    import torch
    from paper_1209_0410_amd import learned
    nq = q.shape[0]
    hq = torch.from_numpy(q).pin_memory()
    hid = torch.empty((nq, k), dtype=torch.int32).pin_memory()
    hd = torch.empty((nq, k), dtype=torch.int32).pin_memory()
    gq = torch.empty((nq, 128), dtype=torch.uint8, device=dev)
    out = (torch.empty((nq, k), dtype=torch.int32, device=dev),
           torch.empty((nq, k), dtype=torch.int32, device=dev))
    feats = torch.empty((nq, learned.FEATURES), dtype=torch.float32, device=dev)
    wq = torch.empty(nq, dtype=torch.int32, device=dev)

    def once():
        gq.copy_(hq, non_blocking=True)
        if model is not None:
            learned.search_learned(ix, model, gq, k, out, sc, feats=feats, w=wq)
        else:
            ix.encode_queries(gq, sc)
            ix.search_encoded(gq, k, w_fix, out, sc, path=forced)
        hid.copy_(out[0], non_blocking=True)
        hd.copy_(out[1], non_blocking=True)

    for _ in range(a.warmup):
        once()
    torch.cuda.synchronize()
    ms = []
    for _ in range(a.steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        once()
        e1.record(stream)
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    med = float(np.median(ms))
    return {"ms": med, "ms_min": float(np.min(ms)), "ms_max": float(np.max(ms)),
            "qps": nq / med * 1e3, "upload_bytes": int(q.nbytes), "download_bytes": 8 * nq * k}


def sub_batch_latency(a, ix, model, gq, k, w_fix, out, sc, stream):
    """Each sub-batch of --latency-batch queries searched alone and timed."""
    import torch
    from paper_1209_0410_amd import learned
    lb = min(a.latency_batch, gq.shape[0])
    lat = []
    for i in range(0, gq.shape[0] - lb + 1, lb) if lb > 0 else []:
        sub = gq[i:i + lb]
        o = (out[0][i:i + lb], out[1][i:i + lb])
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        if model is not None:
            learned.search_learned(ix, model, sub, k, o, sc)
        else:
            ix.search(sub, k, w_fix, out=o, scratch=sc)
        e1.record(stream)
        lat.append((e0, e1))
    torch.cuda.synchronize()
    ms = np.array([e0.elapsed_time(e1) for e0, e1 in lat] or [float("nan")])
    return {"batch": lb, "batches": len(lat), "p50": float(np.percentile(ms, 50)),
            "p99": float(np.percentile(ms, 99))}


def power_leg(a, fn, stream):
    """Socket power and GFX clock while the headline step repeats for
    --power-seconds: amd-smi sampled from a thread (about 3 samples/s),
    samples in the middle of the loop only.  None without amd-smi."""
    import shutil
    import subprocess
    import threading
    import torch
    smi = shutil.which("amd-smi")
    if not smi or a.power_seconds <= 0:
        return None
    samples, stop = [], threading.Event()

    def sampler():
        while not stop.is_set():
            t = time.time()
            try:
                r = subprocess.run([smi, "metric", "-g", "0", "-c", "-p", "--json"],
                                   capture_output=True, text=True, timeout=10)
                d = json.loads(r.stdout)["gpu_data"][0]
                clk = [v["clk"]["value"] for key, v in d["clock"].items()
                       if key.startswith("gfx_") and isinstance(v, dict)
                       and isinstance(v.get("clk"), dict)]
                samples.append((t, float(d["power"]["socket_power"]["value"]),
                                float(np.mean(clk))))
            except Exception:
                pass
            stop.wait(0.2)

    for _ in range(2):
        fn(None, stream)
    torch.cuda.synchronize()
    th = threading.Thread(target=sampler, daemon=True)
    th.start()
    t0 = time.time()
    steps = 0
    while time.time() - t0 < a.power_seconds:
        for _ in range(5):
            fn(None, stream)
        torch.cuda.synchronize()
        steps += 5
    t1 = time.time()
    stop.set()
    th.join()
    mid = [s for s in samples if t0 + 0.5 <= s[0] <= t1 - 0.3]
    if not mid:
        return None
    return {"seconds": t1 - t0, "steps": steps, "ms_per_step": (t1 - t0) / steps * 1e3,
            "samples": len(mid), "socket_power_W": float(np.mean([s[1] for s in mid])),
            "socket_power_W_max": max(s[1] for s in mid),
            "gfx_clock_MHz": float(np.mean([s[2] for s in mid])),
            "gfx_clock_MHz_min": min(s[2] for s in mid)}


def read_probe(a, dev):
    """Achievable streaming-read bandwidth: hc_read_probe over a buffer of
    --probe-gib GiB, median of 5 runs after one warm-up."""
    import torch
    from paper_1209_0410_amd import capi
    from paper_1209_0410_amd.index import _ptr, _stream
    nbytes = a.probe_gib << 30
    buf = torch.ones(nbytes, dtype=torch.uint8, device=dev)
    blocks = 256 * 8
    sink = torch.empty(blocks, dtype=torch.int32, device=dev)
    ms = []
    for i in range(6):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        capi.call("hc_read_probe", _ptr(buf), nbytes, _ptr(sink), blocks, _stream())
        e1.record()
        torch.cuda.synchronize()
        if i:
            ms.append(e0.elapsed_time(e1))
    del buf
    med = float(np.median(ms))
    if a.copy_probe:
        src = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("copy probe: 3 x 1 GiB device-to-device")
    return {"GBs": nbytes / (med * 1e-3) / 1e9, "bytes": nbytes, "runs": len(ms),
            "ms": med, "frac_of_peak": nbytes / (med * 1e-3) / 1e9 / HBM_PEAK_GBS}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def oracle_legs(a, db, q, truth, kt, k, w_fix, fixed_out, learned_out, wv, use_learned, ix,
                rank, gq, dev):
    """(1) The GPU exact kNN against the oracle's on the first --truth-check
    evaluation queries and on 64 training queries, and the GPU labels of those
    training queries against the oracle's.  (2) The oracle's search timed on
    the host cores on a bounded sample of the batch with the headline method's
    w (all threads, then one thread); its results must equal the timed GPU
    step's on every sampled query."""
    import torch
    import oracle
    from paper_1209_0410_amd import datagen, learned
    from paper_1209_0410_amd.index import brute_force
    m = min(a.truth_check, q.shape[0])
    t0 = time.time()
    rid, _ = oracle.brute_force(db, q[:m], kt)
    if not (rid == truth[:m]).all():
        raise AssertionError("GPU exact kNN differs from the oracle on evaluation queries")
    log(f"GPU exact kNN equals the oracle's on {m} evaluation queries "
        f"({time.time() - t0:.1f}s)")
    t0 = time.time()
    oix = oracle.Index(db)
    build = time.time() - t0
    log(f"oracle index over {db.shape[0]} rows built in {build:.1f}s")
    check = {"eval_queries": m}
    if a.train and k <= 16:
        mt = 64
        tq = datagen.make_queries(mt, seed=datagen.SEED_TRAIN)
        gtq = torch.from_numpy(tq).to(dev)
        gt, _ = brute_force(ix.db, gtq, k)
        glab = u32(learned.labels(ix, rank, gtq, gt))
        ot, _ = oracle.brute_force(db, tq, k)
        if not (ot == u32(gt)).all():
            raise AssertionError("GPU exact kNN differs from the oracle on training queries")
        olab = oix.labels(tq, k, ot)
        if not (olab == glab).all():
            raise AssertionError("GPU labels differ from the oracle's")
        log(f"GPU exact kNN and labels equal the oracle's on {mt} training queries")
        check["train_queries"] = mt
    w_of = (lambda s: wv[:s]) if use_learned else (lambda s: w_fix)
    gpu = learned_out if use_learned else fixed_out
    threads = oracle.threads()
    t0 = time.time()
    probe = 16
    oix.search(q[:probe], k, w_of(probe))
    per = (time.time() - t0) / probe
    sample = int(min(len(q), max(probe, a.cpu_seconds / max(per, 1e-9))))
    t0 = time.time()
    sid, sd = oix.search(q[:sample], k, w_of(sample))
    dt = time.time() - t0
    if not ((gpu[0][:sample] == sid).all() and (gpu[1][:sample] == sd).all()):
        raise AssertionError("the timed GPU step differs from the oracle on the sample")
    log(f"timed GPU step equals the oracle on all {sample} sampled queries "
        f"({sample / dt:.1f} q/s on {threads} threads)")
    if use_learned:                 # the fixed-w step too, on a few queries
        s2 = min(32, len(q))
        fid, fd = oix.search(q[:s2], k, w_fix)
        if not ((fixed_out[0][:s2] == fid).all() and (fixed_out[1][:s2] == fd).all()):
            raise AssertionError("the fixed-w GPU step differs from the oracle")
        check["fixed_w_queries"] = s2
    oracle.set_threads(1)
    try:
        s1 = int(min(sample, max(4, a.cpu_seconds_1t / max(per * threads, 1e-9))))
        t0 = time.time()
        sid1, sd1 = oix.search(q[:s1], k, w_of(s1))
        dt1 = time.time() - t0
        t1 = oracle.threads()
    finally:
        oracle.set_threads(threads)
    assert (sid1 == sid[:s1]).all() and (sd1 == sd[:s1]).all()
    log(f"oracle on 1 thread: {s1 / dt1:.2f} q/s ({s1} queries)")
    check["sample_queries"] = sample
    what = "learned per-query w" if use_learned else f"fixed w={w_fix}"
    cpu = {"value": sample / dt, "unit": "queries/s", "cores": threads, "kind": "oracle",
           "sample": f"first {sample} of the {len(q)} evaluation queries, {what}, k={k}, "
                     f"N={db.shape[0]}; the oracle's own index, built in {build:.1f}s (not "
                     f"timed); its results equal the timed GPU step's on all of them",
           "threads_all": {"threads": threads, "value": sample / dt, "queries": sample},
           "threads_1": {"threads": t1, "value": s1 / dt1, "queries": s1},
           "cpu_model": cpu_model(), "nproc": os.cpu_count()}
    del oix
    return check, cpu


# ---------------------------------------------------------------------------
# secondary legs on the first --secondary-n rows
# ---------------------------------------------------------------------------

def run_secondary(a, gdb_all, db, k, dev, stream):
    import torch
    from paper_1209_0410_amd import datagen, learned
    from paper_1209_0410_amd.index import Index, brute_force
    n2 = a.secondary_n
    gdb = gdb_all[:n2]
    t0 = time.time()
    ix = Index(gdb)
    torch.cuda.synchronize()
    build_s = time.time() - t0
    rank = learned.ranks(ix)
    if a.rowstore:
        ix.attach_rowstore()
    nq = 100_000
    q = datagen.make_queries(nq)                   # the plain-method batch (seed 2)
    gq = torch.from_numpy(q).to(dev)
    sc = ix.scratch(nq, k)
    out = (torch.empty((nq, k), dtype=torch.int32, device=dev),
           torch.empty((nq, k), dtype=torch.int32, device=dev))
    rq = 10_000
    kt = min(k, 10)
    truth = u32(brute_force(gdb, gq[:rq].contiguous(), kt)[0])
    if a.cpu_baseline:
        import oracle
        m = min(a.truth_check, rq)
        rid, _ = oracle.brute_force(db[:n2], q[:m], kt)
        if not (rid == truth[:m]).all():
            raise AssertionError("GPU exact kNN differs from the oracle (secondary)")
        log(f"N={n2}: GPU exact kNN equals the oracle's on {m} queries")
    work = Work(ix, rank, gq, k)
    forced = {"auto": 0, "gather": 1, "band": 2}[a.path]

    def rec():
        return learned.recall_at_k(u32(out[0][:rq]), truth)

    sweep = []
    for w in sorted({int(x) for x in a.sweep.split(",") if x}):
        t = summary(timed(fixed_step(ix, gq, k, w, out, sc, forced), a.sweep_steps, 1, stream,
                          warm_s=0.25))
        p = path_name(forced if forced else ix.path(nq, k, w, sc.numel()))
        wk = work.of(w=w)
        roof = roofline_of(p, wk, t["main_kernel_ms"])
        row = dict(w=w, path=p, **t, qps=nq / t["step_ms"] * 1e3, recall=rec(),
                   union_per_query=wk["union_per_query"], roofline=roof)
        sweep.append(row)
        log(f"N={n2} w={w} ({p}): {t['step_ms']:.3f} ms/step, recall {row['recall']:.4f}, "
            f"{roof['achieved']:.0f} {roof['unit']} ({roof['frac']:.1%} of {roof['bound']})")
    cq = datagen.make_queries(a.calib_q, seed=datagen.SEED_CALIB)
    gcq = torch.from_numpy(cq).to(dev)
    ctruth, _ = brute_force(gdb, gcq, kt)
    w_c, rec_c = learned.calibrate_fixed_w(ix, gcq, ctruth, k, CALIB_TARGET, hi=1 << 17)
    t = summary(timed(fixed_step(ix, gq, k, w_c, out, sc, forced), a.steps, a.warmup, stream))
    p = path_name(forced if forced else ix.path(nq, k, w_c, sc.numel()))
    wk = work.of(w=w_c)
    tb, tsrc = counted_traffic(f"n={n2} nq={nq} k={k} w={w_c}", "band" if p == "band"
                               else "gather")
    roof = roofline_of(p, wk, t["main_kernel_ms"], tb)
    if tsrc:
        roof["traffic_source"] = tsrc
    c2 = dict(n=n2, nq=nq, w=w_c, calib_recall=rec_c, path=p, **t,
              qps=nq / t["step_ms"] * 1e3, recall=rec(), union_per_query=wk["union_per_query"],
              roofline=roof)
    log(f"N={n2} fixed w={w_c} at recall {c2['recall']:.4f}: {t['step_ms']:.3f} ms/step, "
        f"{c2['qps']:.3e} q/s, main kernel {t['main_kernel_ms']:.3f} ms "
        f"({roof['frac']:.1%} of {roof['bound']})")
    res = {"n": n2, "build_s": build_s, "sweep": sweep, "fixed_w_at_recall": c2}
    if a.uneven:
        res["uneven"] = run_uneven(a, ix, rank, gdb, dev)
    if a.f4:
        res["f4"] = run_f4(a, ix, gdb, gq, gcq, ctruth, out, rec, w_c, build_s, stream)
    del ix
    return res


def run_f4(a, ix, gdb, gq, gcq, ctruth, out, rec, w_fix, build_s, stream):
    """The Z-order curve in place of the Hilbert curve (same data, same
    calibration), and rows appended to a built index without a rebuild."""
    import torch
    from paper_1209_0410_amd import learned
    from paper_1209_0410_amd.index import Index
    k = a.k
    nq = gq.shape[0]
    zx = Index(gdb, curve="zorder")
    zsc = zx.scratch(nq)

    def step(w):
        def fn(ev, st):
            if ev:
                ev[0].record(st)
                ev[1].record(st)
            zx.search(gq, k, w, out=out, scratch=zsc)
            if ev:
                ev[2].record(st)
        return fn

    timed(step(w_fix), 1, 1, stream)
    rec_h_w = rec()
    w_z, rec_c = learned.calibrate_fixed_w(zx, gcq, ctruth, k, CALIB_TARGET, hi=1 << 20)
    t = summary(timed(step(w_z), a.steps, a.warmup, stream))
    z = dict(recall_at_hilbert_w=rec_h_w, hilbert_w=w_fix, w=w_z, calib_recall=rec_c,
             step_ms=t["step_ms"], qps=nq / t["step_ms"] * 1e3, recall=rec())
    log(f"z-order: recall {rec_h_w:.4f} at the Hilbert w={w_fix}; needs w={w_z}: "
        f"{t['step_ms']:.3f} ms/step, recall {z['recall']:.4f}")
    del zx, zsc
    n = gdb.shape[0]
    m = max(1, n // 100)
    base = Index(gdb[:n - m])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ins = base.insert(gdb)
    torch.cuda.synchronize()
    ins_s = time.perf_counter() - t0
    same = all(torch.equal(ins.curve(c)[0], ix.curve(c)[0]) and
               torch.equal(ins.curve(c)[1], ix.curve(c)[1]) for c in range(8))
    log(f"insert {m} rows into {n - m}: {ins_s:.3f}s (full build {build_s:.3f}s), "
        f"equal to the full build: {same}")
    del base, ins
    return {"zorder": z, "insert": dict(n0=n - m, m=m, insert_s=ins_s, full_build_s=build_s,
                                        equals_full_build=bool(same))}


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
    cfg, entry = Tuner().best(ix, gq, gw, gk, sample=nq)
    log(f"uneven: tuned {entry['tried']} shapes in {time.time() - t0:.1f}s: "
        f"chunk={cfg.chunk_slots} split={cfg.max_split} per_cu={cfg.blocks_per_cu} "
        f"({entry['ms']:.3f} ms vs default {entry['default_ms']:.3f} ms)")
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
    ms_all = [e0.elapsed_time(e1) for e0, e1 in ev]
    ms = float(np.median(ms_all))
    uni = int(u32(learned.union_sizes(ix, rank, gq, 0, gw)).astype(np.int64).sum())
    pos = u32(ix.positions(gq)).astype(np.int64)
    wl = w.astype(np.int64)[:, None]
    slots = int((np.minimum(pos + wl, ix.n) - np.maximum(pos - wl, 0)).sum())
    ab = 4 * slots + 128 * uni + 8 * int(k.sum())
    m = min(nq, 2000)
    truth = u32(brute_force(gdb, gq[:m].contiguous(), 10)[0])
    got = u32(out[0][:m])
    hits = [len(set(got[i, :min(int(k[i]), 10)].tolist()) &
                set(truth[i, :min(int(k[i]), 10)].tolist())) / min(int(k[i]), 10)
            for i in range(m)]
    ach = ab / (ms * 1e-3) / 1e9
    row = dict(nq=nq, ms_per_batch=ms, ms_min=float(np.min(ms_all)),
               ms_max=float(np.max(ms_all)), qps=nq / ms * 1e3, mean_w=float(w.mean()),
               k_mix={str(v): int((k == v).sum()) for v in np.unique(k)},
               cfg=[cfg.chunk_slots, cfg.max_split, cfg.blocks_per_cu], tune=entry,
               union_per_query=uni / nq, alg_bytes=ab,
               roofline={"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": ach / HBM_PEAK_GBS,
                         "kernel": "whole graph replay (k_items dominant)"},
               recall_at_min_k_10=float(np.mean(hits)), graph=True)
    log(f"uneven: {ms:.3f} ms per batch of {nq}, {row['qps']:.3e} q/s, {ach:.0f} GB/s, "
        f"recall@min(k,10) {row['recall_at_min_k_10']:.4f}")
    return row


if __name__ == "__main__":
    main()
