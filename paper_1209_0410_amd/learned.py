"""Learned probe depth: labels, features, an MLP trained on the GPU, and the
per-query w it predicts.

The paper uses one probe depth for every query.  Here each query gets its own
window w = clamp(ceil(2^(y + delta))), y = MLP(features), trained to estimate
log2 of the query's label (the smallest w whose candidate union holds its
exact top-k).  Every computation runs in libhypercurves.so (hc_features,
hc_labels, hc_mlp_*, hc_adam_step); this module allocates tensors, sequences
the calls and draws the seeded batch order.
"""
import ctypes as ct
import math

import numpy as np
import torch

from . import capi
from .index import Index, _empty_bytes, _ptr, _stream, _check_rows

FEATURES = 24
NPARAMS = 5825
DIMS = (24, 64, 64)


def _layers():
    i, h1, h2 = DIMS
    return [(h1, i), (h1,), (h2, h1), (h2,), (h2,), (1,)]


def init_params(seed: int) -> np.ndarray:
    """He-uniform weights (bound sqrt(6 / fan_in)), zero biases, float32."""
    rng = np.random.default_rng(seed)
    out = []
    fan = {0: DIMS[0], 2: DIMS[1], 4: DIMS[2]}
    for li, shape in enumerate(_layers()):
        if li in fan:
            b = math.sqrt(6.0 / fan[li])
            out.append(rng.uniform(-b, b, size=int(np.prod(shape))))
        else:
            out.append(np.zeros(int(np.prod(shape))))
    p = np.concatenate(out).astype(np.float32)
    assert p.size == NPARAMS
    return p


def ranks(ix: Index):
    """int32 (n, curves): place of every id in every list."""
    r = torch.empty((ix.n, ix.curves), dtype=torch.int32, device=ix.db.device)
    capi.call("hc_index_ranks", ix.handle, _ptr(r), _stream())
    return r


def labels(ix: Index, rank, queries, truth_ids):
    _check_rows(queries, "queries")
    nq, k = truth_ids.shape
    out = torch.empty(nq, dtype=torch.int32, device=queries.device)
    sc = ix.scratch(nq)
    capi.call("hc_labels", ix.handle, _ptr(rank), _ptr(queries), nq, k, _ptr(truth_ids),
              _ptr(out), _ptr(sc), sc.numel(), _stream())
    return out


def mixed_k_examples(ix: Index, rank, db, queries, ks):
    """Features (with each query's own k) and labels (the smallest w that
    recovers its exact top-k) for queries with per-query k (1 <= k <= 16):
    training examples for requests of mixed depth."""
    from .index import brute_force
    ks = np.asarray(ks, np.uint32)
    gk = torch.from_numpy(ks.view(np.int32)).to(queries.device)
    feats = features(ix, queries, 0, gk)
    labs = torch.empty(queries.shape[0], dtype=torch.int32, device=queries.device)
    for k in np.unique(ks):
        m = torch.from_numpy(np.nonzero(ks == k)[0]).to(queries.device)
        sub = queries[m].contiguous()
        truth, _ = brute_force(db, sub, int(k))
        labs[m] = labels(ix, rank, sub, truth)
    return feats, labs


def union_sizes(ix: Index, rank, queries, w=0, w_per_query=None):
    _check_rows(queries, "queries")
    nq = queries.shape[0]
    out = torch.empty(nq, dtype=torch.int32, device=queries.device)
    sc = ix.scratch(nq)
    capi.call("hc_union_sizes", ix.handle, _ptr(rank), _ptr(queries), nq, int(w),
              _ptr(w_per_query) if w_per_query is not None else None, _ptr(out), _ptr(sc),
              sc.numel(), _stream())
    return out


def features(ix: Index, queries, k=10, k_per_query=None):
    """float32 (nq, 24)."""
    _check_rows(queries, "queries")
    nq = queries.shape[0]
    out = torch.empty((nq, FEATURES), dtype=torch.float32, device=queries.device)
    sc = ix.scratch(nq)
    capi.call("hc_features", ix.handle, _ptr(queries), nq, int(k),
              _ptr(k_per_query) if k_per_query is not None else None, _ptr(out), _ptr(sc),
              sc.numel(), _stream())
    return out


def to_bf16(x):
    out = torch.empty(x.numel(), dtype=torch.int16, device=x.device)
    capi.call("hc_to_bf16", _ptr(x), x.numel(), _ptr(out), _stream())
    return out


class WModel:
    """The probe-depth MLP: FP32 master weights, BF16 compute copy, the feature
    standardisation and the calibrated offset delta."""

    def __init__(self, device, seed=0, w_min=8, w_max=1 << 17):
        self.device = device
        self.master = torch.from_numpy(init_params(seed)).to(device)
        self.bf16 = to_bf16(self.master)
        self.norm = torch.cat([torch.zeros(FEATURES), torch.ones(FEATURES)]).to(device)
        self.delta = 0.0
        self.w_min, self.w_max = int(w_min), int(w_max)
        self.w_hint = 64        # typical predicted w (sizes the search's execution path)
        self.confidence = 1.0   # weight of the prediction against the training mean
        self.y_mean = 0.0       # mean of the training targets

    def targets(self, label):
        """y = log2(clamp(label, w_min, w_max)) as float32 (hc_mlp_targets)."""
        label = label.contiguous()
        y = torch.empty(label.shape[0], dtype=torch.float32, device=label.device)
        capi.call("hc_mlp_targets", _ptr(label), label.shape[0], self.w_min, self.w_max,
                  _ptr(y), _stream())
        return y

    def set_norm(self, feats):
        """Standardisation from training features (hc_feature_norm); a feature
        that does not vary in training keeps unit scale (so unseen values stay
        moderate)."""
        feats = feats.contiguous()
        norm = torch.empty(2 * FEATURES, dtype=torch.float32, device=feats.device)
        capi.call("hc_feature_norm", _ptr(feats), feats.shape[0], _ptr(norm), _stream())
        self.norm = norm

    def train(self, feats, y, epochs=20, batch=4096, lr=1e-3, seed=0, log=None):
        """Adam on the MSE of y, batches drawn in a seeded order; returns losses."""
        feats = feats.contiguous()
        y = y.contiguous()
        rows = feats.shape[0]
        sz = ct.c_size_t()
        capi.call("hc_mlp_train_scratch_bytes", batch, ct.byref(sz))
        sc = _empty_bytes(sz.value, self.device)
        grad = torch.zeros(NPARAMS, dtype=torch.float32, device=self.device)
        m = torch.zeros_like(grad)
        v = torch.zeros_like(grad)
        loss = torch.zeros(1, dtype=torch.float32, device=self.device)
        rng = np.random.default_rng(seed)
        self.y_mean = float(np.mean(y.cpu().numpy(), dtype=np.float64))
        t = 0
        losses = []
        for ep in range(epochs):
            order = torch.from_numpy(rng.permutation(rows).astype(np.int32)).to(self.device)
            ep_loss = []
            for b0 in range(0, rows - batch + 1, batch):
                idx = order[b0:b0 + batch]
                capi.call("hc_mlp_backward", _ptr(self.bf16), _ptr(self.norm), _ptr(feats),
                          _ptr(y), _ptr(idx), batch, _ptr(grad), _ptr(loss), _ptr(sc),
                          sc.numel(), _stream())
                t += 1
                capi.call("hc_adam_step", _ptr(self.master), _ptr(m), _ptr(v), _ptr(grad),
                          NPARAMS, t, lr, 0.9, 0.999, 1e-8, _ptr(self.bf16), _stream())
                ep_loss.append(loss.clone())
            losses.append(float(torch.stack(ep_loss).mean()))
            if log:
                log(f"epoch {ep} loss {losses[-1]:.4f}")
        return losses

    def set_confidence(self, lam):
        """Inference weights whose output is y_mean + lam * (y - y_mean): the
        last layer is linear, so its weights are scaled by lam and its bias
        moved toward the training mean (lam = 1: the trained network; lam = 0:
        one w for every query, 2^(y_mean + delta)).  A prediction that carries
        little information about the labels is worth less than its spread
        costs; the calibration picks lam."""
        lam = float(lam)
        p = self.master.detach().cpu().numpy().astype(np.float64).copy()
        w3 = slice(NPARAMS - 1 - DIMS[2], NPARAMS - 1)
        p[w3] *= lam
        p[NPARAMS - 1] = lam * p[NPARAMS - 1] + (1.0 - lam) * self.y_mean
        self.bf16 = to_bf16(torch.from_numpy(p.astype(np.float32)).to(self.device))
        self.confidence = lam

    def predict(self, feats):
        """y = MLP(standardised features), float32 (nq,)."""
        nq = feats.shape[0]
        y = torch.empty(nq, dtype=torch.float32, device=self.device)
        capi.call("hc_mlp_forward", _ptr(self.bf16), _ptr(self.norm), _ptr(feats.contiguous()),
                  None, nq, _ptr(y), _stream())
        return y

    def windows(self, feats, delta=None, w_fallback=64):
        """Per-query w (int32) from the features."""
        nq = feats.shape[0]
        w = torch.empty(nq, dtype=torch.int32, device=self.device)
        d = self.delta if delta is None else delta
        capi.call("hc_mlp_infer", _ptr(self.bf16), _ptr(self.norm), _ptr(feats.contiguous()),
                  nq, float(d), self.w_min, self.w_max, int(w_fallback), _ptr(w), None,
                  _stream())
        return w

    def state(self):
        return {"master": self.master.cpu().numpy(), "norm": self.norm.cpu().numpy(),
                "delta": self.delta, "w_min": self.w_min, "w_max": self.w_max,
                "confidence": self.confidence, "y_mean": self.y_mean}

    def load_state(self, st):
        self.master = torch.from_numpy(np.asarray(st["master"], np.float32)).to(self.device)
        self.bf16 = to_bf16(self.master)
        self.norm = torch.from_numpy(np.asarray(st["norm"], np.float32)).to(self.device)
        self.delta = float(st["delta"])
        self.w_min, self.w_max = int(st["w_min"]), int(st["w_max"])
        self.y_mean = float(st.get("y_mean", 0.0))
        self.set_confidence(st.get("confidence", 1.0))


def recall_at_k(ids, truth):
    """Mean of |approx ∩ exact| / k over the queries (numpy uint32 arrays)."""
    k = truth.shape[1]
    ids = np.asarray(ids, np.uint32)[:, :k]
    truth = np.asarray(truth, np.uint32)
    # ids within a row are distinct (as are the truth's), so each match counts once
    hit = (ids[:, :, None] == truth[:, None, :]).any(axis=2) & (ids != 0xFFFFFFFF)
    return float(hit.sum(axis=1).mean()) / k


def quick_path(ix: Index, nq, k, w):
    """The faster execution path for a calibration batch: banded when each list
    entry lies in several of the batch's windows (k <= 16, or up to
    HC_BAND_K_MAX with the row store attached), whatever the block
    count (both paths give the same results; the automatic choice also wants
    enough blocks to fill the device, which a small batch lacks)."""
    band_k = k <= 16 or (k <= capi.HC_BAND_K_MAX and getattr(ix, "rowstore", None) is not None)
    return capi.HC_PATH_BAND if (band_k and 2.0 * w * nq >= 3.5 * ix.n) else capi.HC_PATH_GATHER


def calibrate_delta(ix: Index, model: WModel, queries, feats, truth, k, target=0.90,
                    lo=-4.0, hi=8.0, iters=12):
    """Smallest delta (bisection) whose searches reach mean recall@k >= target."""
    truth_np = truth.cpu().numpy().view(np.uint32)
    nq = queries.shape[0]

    def rec(d):
        w = model.windows(feats, d)
        wm = int(w.float().mean().item()) or 64
        ids, _ = ix.search(queries, k, wm, w_per_query=w, path=quick_path(ix, nq, k, wm))
        return recall_at_k(ids.cpu().numpy().view(np.uint32), truth_np)

    if rec(hi) < target:
        lo = hi
    else:
        for _ in range(iters):
            mid = 0.5 * (lo + hi)
            if rec(mid) >= target:
                hi = mid
            else:
                lo = mid
    model.w_hint = max(1, int(model.windows(feats, hi).float().mean().item()))
    return hi, rec(hi)


def search_learned(ix: Index, model: WModel, queries, k, out, scratch, feats=None, w=None,
                   w_fallback=64):
    """One pass of the learned-w search: features (which also leave the query
    keys in `scratch`), the MLP's w per query, then the search itself on those
    keys.  Returns (ids, dists, w)."""
    nq = queries.shape[0]
    if feats is None:
        feats = torch.empty((nq, FEATURES), dtype=torch.float32, device=queries.device)
    if w is None:
        w = torch.empty(nq, dtype=torch.int32, device=queries.device)
    capi.call("hc_features", ix.handle, _ptr(queries), nq, int(k), None, _ptr(feats),
              _ptr(scratch), scratch.numel(), _stream())
    capi.call("hc_mlp_infer", _ptr(model.bf16), _ptr(model.norm), _ptr(feats), nq,
              float(model.delta), model.w_min, model.w_max, int(w_fallback), _ptr(w), None,
              _stream())
    ix.search_encoded(queries, k, model.w_hint, out, scratch, w_per_query=w)
    return out[0], out[1], w


def calibrate_fixed_w(ix: Index, queries, truth, k, target=0.90, lo=1, hi=1 << 17):
    """Smallest fixed w (bisection on integers) whose search reaches mean
    recall@k >= target; the recall never drops as w grows (the candidate sets
    are nested and every true neighbour found stays among the k nearest)."""
    truth_np = truth.cpu().numpy().view(np.uint32)
    nq = queries.shape[0]

    def rec(w):
        ids, _ = ix.search(queries, k, int(w), path=quick_path(ix, nq, k, w))
        return recall_at_k(ids.cpu().numpy().view(np.uint32), truth_np)

    if rec(hi) < target:
        return hi, rec(hi)
    while hi - lo > max(1, lo // 64):     # about 1.5% resolution
        mid = (lo + hi) // 2
        if rec(mid) >= target:
            hi = mid
        else:
            lo = mid + 1
    return hi, rec(hi)
