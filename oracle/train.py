"""FP64 oracle of one training step of the localization network -- TEST
INFRASTRUCTURE ONLY (same rules as the rest of ``oracle``: only tests,
smoke() and the bench's CPU leg use it; it never touches the product path).

The paper trains its network with DECODE's loss plus a binary cross-entropy
on the per-pixel detection probability (Sec. 3.3: the cross-entropy of
predicted and true occupancy, together with the counting loss, constrains the
whole distribution of molecules).  Written out here for the residual network
with the 10-output head (probability, offsets, their uncertainties), per
frame of P = h w pixels with maps m (logit l, dx, dy, dz, ph, raw sigmas
u_x, u_y, u_z, u_N, background) and its true emitters e = 1 .. E:

  p_k = sigmoid(l_k); y_k = 1 iff a true emitter lies in pixel k
  L_bce   = (1/P) sum_k [softplus(l_k) - y_k l_k]                 (BCE on l)
  mu = sum_k p_k,  v = sum_k p_k (1 - p_k) + 1e-4
  L_count = log(2 pi v) / 2 + (E - mu)^2 / (2 v)       (Gaussian count model)
  m_k = (col + 0.5 + dx, row + 0.5 + dy, dz, ph),  s_kd = softplus(u_kd) + 0.01
  q_ek = log p_k - log mu + sum_d log N(t_ed; m_kd, s_kd^2)
  L_loc   = -sum_e logsumexp_k q_ek        (mixture over pixels, weights p/mu)
  L_frame = L_bce + L_count + L_loc;  the batch loss is the mean over frames.

t_e = (x, y, z / z_scale, photons / ph_scale) of emitter e.  Gradients are
taken by hand, layer by layer, in the order of the definitions (the network's
backward pass is plain convolutions: the transposed 3x3 convolution is the
forward one with flipped, transposed weights; weight gradients are sums of
products over pixels), for the residual network and for the
dense-connection network (its backward pass through the concatenation).
"""
from __future__ import annotations

import math
from typing import Dict, List, Tuple

import numpy as np

from . import conv3x3, preprocess, sigma_of, softplus

VAR_EPS = 1e-4


def _sig(v):
    return 0.5 * (1.0 + np.tanh(0.5 * v))


def _log_sig(v):
    """log sigmoid(v) = -softplus(-v)."""
    return -softplus(-v)


def occupancy(truth, h: int, w: int) -> np.ndarray:
    """y[h][w]: 1 where a true emitter's (x, y) falls in the pixel."""
    y = np.zeros((h, w), np.float64)
    for t in truth:
        r, c = int(math.floor(t["y"])), int(math.floor(t["x"]))
        if 0 <= r < h and 0 <= c < w:
            y[r, c] = 1.0
    return y


def frame_loss(maps: np.ndarray, truth, spec) -> Tuple[Dict[str, float], np.ndarray]:
    """Loss of one frame and its gradient with respect to the maps [10][h][w]."""
    nh, h, w = maps.shape
    assert nh == 10
    P = h * w
    l = maps[0]
    p = _sig(l)
    g = np.zeros_like(maps)
    # binary cross-entropy on the logit
    yk = occupancy(truth, h, w)
    L_bce = float(np.sum(softplus(l) - yk * l)) / P
    g[0] += (p - yk) / P
    # count
    E = len(truth)
    mu = float(np.sum(p))
    v = float(np.sum(p * (1 - p))) + VAR_EPS
    L_cnt = 0.5 * math.log(2 * math.pi * v) + (E - mu) ** 2 / (2 * v)
    dmu = -(E - mu) / v
    dv = 1 / (2 * v) - (E - mu) ** 2 / (2 * v * v)
    g[0] += p * (1 - p) * (dmu + (1 - 2 * p) * dv)
    # localisation: a mixture over pixels
    L_loc = 0.0
    if E:
        rows, cols = np.mgrid[0:h, 0:w].astype(np.float64)
        mean = [cols + 0.5 + maps[1], rows + 0.5 + maps[2], maps[3], maps[4]]
        s = [sigma_of(maps[5 + d]) for d in range(4)]
        logw = _log_sig(l) - math.log(mu)
        for t in truth:
            tv = [t["x"], t["y"], t["z_nm"] / spec.z_scale, t["photons"] / spec.ph_scale]
            q = logw.copy()
            for d in range(4):
                q += -0.5 * math.log(2 * math.pi) - np.log(s[d]) - (tv[d] - mean[d]) ** 2 / (2 * s[d] ** 2)
            qmax = float(np.max(q))
            lse = qmax + math.log(float(np.sum(np.exp(q - qmax))))
            L_loc -= lse
            r = np.exp(q - lse)
            # through log p_k and -log mu
            g[0] += -r * (1 - p) + p * (1 - p) / mu
            for d in range(4):
                g[1 + d] += -r * (tv[d] - mean[d]) / s[d] ** 2
                g[5 + d] += -r * (-1 / s[d] + (tv[d] - mean[d]) ** 2 / s[d] ** 3) * _sig(maps[5 + d])
    return {"bce": L_bce, "count": L_cnt, "loc": L_loc, "total": L_bce + L_cnt + L_loc}, g


def _relu(v):
    return np.maximum(v, 0.0)


def _flip_t(W):
    """Weights of the transposed 3x3 convolution: W'[ci][co][u][v] = W[co][ci][2-u][2-v]."""
    return np.ascontiguousarray(W[:, :, ::-1, ::-1].transpose(1, 0, 2, 3))


def _wgrad(dy: np.ndarray, x: np.ndarray, d: int) -> np.ndarray:
    """dW[co][ci][u][v] = sum_ij dy[co][i][j] x[ci][i + d(u-1)][j + d(v-1)] (zero outside)."""
    cin, h, w = x.shape
    xp = np.zeros((cin, h + 2 * d, w + 2 * d))
    xp[:, d:d + h, d:d + w] = x
    out = np.empty((dy.shape[0], cin, 3, 3))
    for u in range(3):
        for v in range(3):
            xs = xp[:, u * d:u * d + h, v * d:v * d + w]
            out[:, :, u, v] = np.tensordot(dy, xs, axes=([1, 2], [1, 2]))
    return out


def frame_grads(frame: np.ndarray, truth, spec, wts: Dict[str, np.ndarray], gain=0.5, offset=100.0):
    """Loss of one frame and the gradient of every weight tensor."""
    W = {k: np.asarray(v, np.float64) for k, v in wts.items()}
    x = preprocess(frame[None], gain, offset, spec.in_scale)[0][None]
    a0 = _relu(conv3x3(x, W["stem.w"], W["stem.b"], 1))
    acts = []
    a = a0
    for k, d in enumerate(spec.dilations):
        t = _relu(conv3x3(a, W[f"blk{k}.w1"], W[f"blk{k}.b1"], d))
        an = _relu(conv3x3(t, W[f"blk{k}.w2"], W[f"blk{k}.b2"], d) + a)
        acts.append((a, t, an))
        a = an
    maps = np.tensordot(W["head.w"], a, axes=(1, 0)) + W["head.b"][:, None, None]
    loss, gm = frame_loss(maps, truth, spec)
    G = {}
    G["head.w"] = np.tensordot(gm, a, axes=([1, 2], [1, 2]))
    G["head.b"] = gm.sum(axis=(1, 2))
    da = np.tensordot(W["head.w"], gm, axes=(0, 0))
    for k in reversed(range(len(spec.dilations))):
        d = spec.dilations[k]
        ain, t, an = acts[k]
        du = da * (an > 0)
        G[f"blk{k}.w2"] = _wgrad(du, t, d)
        G[f"blk{k}.b2"] = du.sum(axis=(1, 2))
        ds = conv3x3(du, _flip_t(W[f"blk{k}.w2"]), None, d) * (t > 0)
        G[f"blk{k}.w1"] = _wgrad(ds, ain, d)
        G[f"blk{k}.b1"] = ds.sum(axis=(1, 2))
        da = du + conv3x3(ds, _flip_t(W[f"blk{k}.w1"]), None, d)
    ds0 = da * (a0 > 0)
    G["stem.w"] = _wgrad(ds0, x, 1)
    G["stem.b"] = ds0.sum(axis=(1, 2))
    return loss, G, maps


def _pool2(a: np.ndarray):
    """2 x 2 max pooling of [C][h][w] to [C][ceil(h/2)][ceil(w/2)] (a window at
    an odd edge holds the pixels it has) and each window's argmax: the first
    maximum in the window's raster order (dy, dx)."""
    C, h, w = a.shape
    h2, w2 = (h + 1) // 2, (w + 1) // 2
    pad = np.full((C, 2 * h2, 2 * w2), -np.inf)
    pad[:, :h, :w] = a
    win = pad.reshape(C, h2, 2, w2, 2).transpose(0, 1, 3, 2, 4).reshape(C, h2, w2, 4)
    return win.max(axis=-1), np.argmax(win, axis=-1)


def _pool2_back(g: np.ndarray, idx: np.ndarray, h: int, w: int) -> np.ndarray:
    """The pooling's gradient: each window's gradient goes to its argmax."""
    C, h2, w2 = g.shape
    out = np.zeros((C, 2 * h2, 2 * w2))
    cc, yy, xx = np.meshgrid(np.arange(C), np.arange(h2), np.arange(w2), indexing="ij")
    out[cc, 2 * yy + idx // 2, 2 * xx + idx % 2] = g
    return out[:, :h, :w]


def _up2(v: np.ndarray, h: int, w: int) -> np.ndarray:
    """Nearest upsampling to h x w: out[y][x] = v[y // 2][x // 2]."""
    return v[:, np.arange(h) // 2][:, :, np.arange(w) // 2]


def _up2_back(g: np.ndarray, h2: int, w2: int) -> np.ndarray:
    """The upsampling's gradient: each coarse pixel sums its (up to) four fine ones."""
    C, h, w = g.shape
    pad = np.zeros((C, 2 * h2, 2 * w2))
    pad[:, :h, :w] = g
    return pad.reshape(C, h2, 2, w2, 2).sum(axis=(2, 4))


def dense_frame_grads(frame: np.ndarray, truth, spec, wts: Dict[str, np.ndarray], gain=0.5, offset=100.0):
    """Loss of one frame and the gradient of every weight tensor of the
    dense-connection network (Sec. 3.2.1: each layer of a block reads the
    concatenation of the block input and the earlier layers' outputs; a 1x1
    transition over the whole concatenation gives the block's output).

    Backward through a block: the transition's pre-activation gradient gives
    its weight gradient against the concatenation and the concatenation's
    gradient (the transposed 1x1 map); then, from the last layer to the first,
    a layer's output channels of that gradient, masked where the layer's ReLU
    was off, give the layer's weight gradient against its input (the
    concatenation so far) and add the transposed 3x3 convolution of it to the
    gradient of that input.  The first C channels are then the gradient at the
    block's input.

    With the two-stage U-Net after the blocks (Sec. 3.2: the fine-grained
    stage), its backward runs first: through u0's convolution over [a0,
    up(u1)], the upsampling (each coarse pixel sums the gradients of the fine
    pixels it fills), u1's convolution over [d1, up(d2)], d2's and d1's
    convolutions and the max poolings (a window's gradient goes to its first
    maximum in raster order), and the two paths' gradients at d1 and at a0
    are added."""
    if spec.unet not in (0, 2):
        raise ValueError("the U-Net stage has 0 or 2 levels")
    W = {k: np.asarray(v, np.float64) for k, v in wts.items()}
    C, Gr, L = spec.C, spec.growth, spec.layers
    x = preprocess(frame[None], gain, offset, spec.in_scale)[0][None]
    a0 = _relu(conv3x3(x, W["stem.w"], W["stem.b"], 1))
    a = a0
    blocks = []
    for k, d in enumerate(spec.dilations):
        cat = a
        for i in range(L):
            new = _relu(conv3x3(cat, W[f"blk{k}.l{i}.w"], W[f"blk{k}.l{i}.b"], d))
            cat = np.concatenate([cat, new], axis=0)
        t = _relu(np.tensordot(W[f"blk{k}.t.w"], cat, axes=(1, 0)) + W[f"blk{k}.t.b"][:, None, None])
        blocks.append((cat, t))
        a = t
    if spec.unet:
        ua = a
        h, w = ua.shape[1:]
        h1, w1 = (h + 1) // 2, (w + 1) // 2
        h2, w2 = (h1 + 1) // 2, (w1 + 1) // 2
        p1, i1 = _pool2(ua)
        d1 = _relu(conv3x3(p1, W["unet.d1.w"], W["unet.d1.b"], 1))
        p2, i2 = _pool2(d1)
        d2 = _relu(conv3x3(p2, W["unet.d2.w"], W["unet.d2.b"], 1))
        c1 = np.concatenate([d1, _up2(d2, h1, w1)], axis=0)
        u1 = _relu(conv3x3(c1, W["unet.u1.w"], W["unet.u1.b"], 1))
        c0 = np.concatenate([ua, _up2(u1, h, w)], axis=0)
        a = _relu(conv3x3(c0, W["unet.u0.w"], W["unet.u0.b"], 1))
    maps = np.tensordot(W["head.w"], a, axes=(1, 0)) + W["head.b"][:, None, None]
    loss, gm = frame_loss(maps, truth, spec)
    G = {}
    G["head.w"] = np.tensordot(gm, a, axes=([1, 2], [1, 2]))
    G["head.b"] = gm.sum(axis=(1, 2))
    da = np.tensordot(W["head.w"], gm, axes=(0, 0))
    if spec.unet:
        gu0 = da * (a > 0)
        G["unet.u0.w"] = _wgrad(gu0, c0, 1)
        G["unet.u0.b"] = gu0.sum(axis=(1, 2))
        gc0 = conv3x3(gu0, _flip_t(W["unet.u0.w"]), None, 1)
        gu1 = _up2_back(gc0[C:], h1, w1) * (u1 > 0)
        G["unet.u1.w"] = _wgrad(gu1, c1, 1)
        G["unet.u1.b"] = gu1.sum(axis=(1, 2))
        gc1 = conv3x3(gu1, _flip_t(W["unet.u1.w"]), None, 1)
        gd2 = _up2_back(gc1[C:], h2, w2) * (d2 > 0)
        G["unet.d2.w"] = _wgrad(gd2, p2, 1)
        G["unet.d2.b"] = gd2.sum(axis=(1, 2))
        gd1 = (gc1[:C] + _pool2_back(conv3x3(gd2, _flip_t(W["unet.d2.w"]), None, 1), i2, h1, w1)) * (d1 > 0)
        G["unet.d1.w"] = _wgrad(gd1, p1, 1)
        G["unet.d1.b"] = gd1.sum(axis=(1, 2))
        da = gc0[:C] + _pool2_back(conv3x3(gd1, _flip_t(W["unet.d1.w"]), None, 1), i1, h, w)
    for k in reversed(range(len(spec.dilations))):
        d = spec.dilations[k]
        cat, t = blocks[k]
        gt = da * (t > 0)
        G[f"blk{k}.t.w"] = np.tensordot(gt, cat, axes=([1, 2], [1, 2]))
        G[f"blk{k}.t.b"] = gt.sum(axis=(1, 2))
        gc = np.tensordot(W[f"blk{k}.t.w"], gt, axes=(0, 0))
        for i in reversed(range(L)):
            lo = C + i * Gr
            gl = gc[lo:lo + Gr] * (cat[lo:lo + Gr] > 0)
            G[f"blk{k}.l{i}.w"] = _wgrad(gl, cat[:lo], d)
            G[f"blk{k}.l{i}.b"] = gl.sum(axis=(1, 2))
            gc[:lo] += conv3x3(gl, _flip_t(W[f"blk{k}.l{i}.w"]), None, d)
        da = gc[:C]
    ds0 = da * (a0 > 0)
    G["stem.w"] = _wgrad(ds0, x, 1)
    G["stem.b"] = ds0.sum(axis=(1, 2))
    return loss, G, maps


def batch_grads(frames: np.ndarray, truths: List, spec, wts, gain=0.5, offset=100.0):
    """Mean loss over the frames and the gradients of the mean (the residual or
    the dense-connection network, by the spec's type)."""
    n = len(frames)
    tot, G = None, None
    fg = dense_frame_grads if hasattr(spec, "growth") else frame_grads
    for f in range(n):
        L, g, _ = fg(frames[f], truths[f], spec, wts, gain, offset)
        tot = dict(L) if tot is None else {k: tot[k] + L[k] for k in tot}
        G = g if G is None else {k: G[k] + g[k] for k in G}
    return {k: v / n for k, v in tot.items()}, {k: v / n for k, v in G.items()}
