"""Training and evaluation of the tile-occupancy gate on the GPU.

Every arithmetic step runs in libdloc's kernels: 4x4 pooling with the
handle's own preprocessing (``dl_gate_pool_net``), forward
(``dl_gate_forward``), binary cross-entropy (``dl_gate_bce``, paper Sec. 3.3),
backward (``dl_gate_backward``, fixed-order reductions) and Adam
(``dl_gate_adam``).  This module only moves data:
generating labelled tiles, shuffling mini-batches and bookkeeping.

Labels: a 256^2 tile is positive iff the ungated localization network emits at
least one emitter in it (the network being gated judges what the gate may
skip).  Training tiles come from frames seeded separately from the evaluation
frames.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Tuple

import numpy as np

from . import GATE_NPARAM, GATE_TILE, Net, emitters_from_device, gate_adam, gate_backward, gate_bce, \
    gate_forward


def tile_counts(rec: np.ndarray, n: int, h: int, w: int) -> np.ndarray:
    """Emitter records per 256^2 tile (tiles frame-major, then row-major)."""
    gy, gx = h // GATE_TILE, w // GATE_TILE
    cnt = np.zeros(n * gy * gx, np.float32)
    if len(rec):
        t = rec["frame"].astype(np.int64) * gy * gx + (rec["row"] // GATE_TILE) * gx + rec["col"] // GATE_TILE
        np.add.at(cnt, t, 1.0)
    return cnt


def tile_labels(rec: np.ndarray, n: int, h: int, w: int) -> np.ndarray:
    """1.0 for every 256^2 tile holding at least one emitter record, else 0.0
    (tiles frame-major, then row-major)."""
    return (tile_counts(rec, n, h, w) > 0).astype(np.float32)


def labelled_tiles(net: Net, frames_iter, device, with_counts=False):
    """Pool every frame batch into gate tiles with ``net``'s own preprocessing
    (its scalars or camera maps, as its gated runs pool them) and label them
    with its own (ungated) detections.  frames_iter yields uint16 numpy
    batches [n][h][w].  with_counts: also return the number of detections per
    tile."""
    import torch
    pooled, labels, counts_ = [], [], []
    for frames in frames_iter:
        n, h, w = frames.shape
        d = torch.from_numpy(np.ascontiguousarray(frames)).to(device)
        cap = max(1024, n * h * w // 64)
        out = torch.empty((cap, 8), dtype=torch.int32, device=device)
        counts = torch.zeros(n + 1, dtype=torch.int32, device=device)
        net.localize_device(d, out, counts)
        p = torch.empty((n * (h // GATE_TILE) * (w // GATE_TILE), 64, 64), dtype=torch.float32, device=device)
        net.gate_pool(d, p)
        torch.cuda.synchronize()
        total = int(counts[n].item())
        rec = emitters_from_device(out, min(total, cap))
        pooled.append(p)
        c = tile_counts(rec, n, h, w)
        counts_.append(c)
        labels.append((c > 0).astype(np.float32))
    out = (torch.cat(pooled), torch.from_numpy(np.concatenate(labels)).to(device))
    return out + (np.concatenate(counts_),) if with_counts else out


@dataclass
class TrainResult:
    theta: np.ndarray
    history: List[Dict[str, float]] = field(default_factory=list)
    val_idx: Optional[np.ndarray] = None


def threshold_at_recall(pooled, labels, theta, idx, target: float = 0.995, counts=None) -> float:
    """Gate probability threshold chosen on held-out tiles: the largest one
    that keeps at least ``target`` of the positive tiles, or, given the
    detections per tile (``counts``), at least ``target`` of the detections."""
    import torch
    g = gate_logits(pooled, theta, idx).astype(np.float64)
    y = labels.index_select(0, torch.from_numpy(np.asarray(idx)).to(labels.device)).cpu().numpy() > 0.5
    wts = None if counts is None else np.asarray(counts, np.float64)[np.asarray(idx)]
    t = threshold_for_recall(g, y, target, wts)
    return float(1.0 / (1.0 + math.exp(-t)))


def train(pooled, labels, theta0: np.ndarray, epochs: int = 20, batch: int = 256, lr: float = 1e-3,
          val_frac: float = 0.1, seed: int = 3005) -> TrainResult:
    """Adam on mean BCE over mini-batches of pooled tiles (torch tensors on the
    GPU); the last ``val_frac`` of a seeded permutation is held out."""
    import torch
    dev = pooled.device
    n = pooled.shape[0]
    rng = np.random.default_rng(seed)
    perm = rng.permutation(n)
    nval = int(round(n * val_frac))
    tr_idx, va_idx = perm[: n - nval], perm[n - nval:]
    theta = torch.from_numpy(np.ascontiguousarray(theta0, np.float32)).to(dev)
    m = torch.zeros_like(theta)
    v = torch.zeros_like(theta)
    grad = torch.empty_like(theta)
    work = torch.empty(batch * GATE_NPARAM, dtype=torch.float32, device=dev)
    logits = torch.empty(batch, dtype=torch.float32, device=dev)
    dlog = torch.empty(batch, dtype=torch.float32, device=dev)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    res = TrainResult(theta=np.asarray(theta0, np.float32), val_idx=va_idx)
    step = 0
    for ep in range(epochs):
        order = tr_idx[rng.permutation(tr_idx.size)]
        tot, nb = 0.0, 0
        for s in range(0, order.size - batch + 1, batch):
            idx = torch.from_numpy(order[s:s + batch]).to(dev)
            xb = pooled.index_select(0, idx)
            yb = labels.index_select(0, idx)
            gate_forward(xb, theta, logits)
            gate_bce(logits, yb, loss, dlog)
            gate_backward(xb, theta, dlog, work, logits, grad)
            step += 1
            gate_adam(theta, m, v, grad, step, lr)
            tot += float(loss.item())
            nb += 1
        ev = evaluate(pooled, labels, theta, va_idx) if nval else {}
        res.history.append({"epoch": ep + 1, "train_loss": tot / max(1, nb), **ev})
    res.theta = theta.cpu().numpy()
    return res


def gate_logits(pooled, theta, idx=None):
    import torch
    dev = pooled.device
    th = theta if isinstance(theta, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(theta, np.float32)).to(dev)
    x = pooled if idx is None else pooled.index_select(0, torch.from_numpy(np.asarray(idx)).to(dev))
    out = torch.empty(x.shape[0], dtype=torch.float32, device=dev)
    for s in range(0, x.shape[0], 4096):
        gate_forward(x[s:s + 4096], th, out[s:s + 4096])
    torch.cuda.synchronize()
    return out.cpu().numpy()


def evaluate(pooled, labels, theta, idx) -> Dict[str, float]:
    """Validation loss, accuracy and, at the 0.05 threshold, tile recall and skip fraction."""
    import torch
    g = gate_logits(pooled, theta, idx).astype(np.float64)
    y = labels.index_select(0, torch.from_numpy(np.asarray(idx)).to(labels.device)).cpu().numpy().astype(np.float64)
    L = float(np.mean(np.maximum(g, 0) - g * y + np.log1p(np.exp(-np.abs(g)))))
    p = 1 / (1 + np.exp(-g))
    keep = p > 0.05
    pos = y > 0.5
    return {"val_loss": L, "val_acc": float(np.mean((p > 0.5) == pos)),
            "val_tile_recall@0.05": float(keep[pos].mean()) if pos.any() else 1.0,
            "val_skip@0.05": float(1 - keep.mean())}


def threshold_for_recall(scores: np.ndarray, positive: np.ndarray, target: float, weights=None) -> float:
    """Largest threshold t such that the positives with score > t carry at
    least ``target`` of the positives' total weight (unit weights: the
    fraction of positive tiles; detection counts: the fraction of detections).
    The positives given up are the lowest-scored ones."""
    sp = scores[positive]
    if sp.size == 0:
        return float(np.max(scores)) + 1.0
    wp = np.ones_like(sp) if weights is None else np.asarray(weights, np.float64)[positive]
    order = np.argsort(sp, kind="stable")
    sp, wp = sp[order], wp[order]
    lose = np.cumsum(wp) <= (1.0 - target) * wp.sum() + 1e-12   # prefix we may give up
    k = int(np.count_nonzero(lose))                          # positives with score < t
    if k >= sp.size:
        return float(sp[-1])
    return float(np.nextafter(sp[k], -np.inf))
