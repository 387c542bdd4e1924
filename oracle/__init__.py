"""FP64 CPU oracle of the localization path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never imports, links or executes anything here, and this
package never imports the product path; the two share only the seeded input
generators in ``smlm_synth``.

The arithmetic lives in ``oracle.c`` (plain C, double precision, loops in the
order of the definition).  This module compiles it with gcc and wraps it with
ctypes, plus the few steps that are plain bookkeeping (record assembly).

Definitions followed (paper Sec. 2.2, Sec. 3.2, Sec. 3.2.1, Sec. 3.3):
see the header of ``oracle.c``, which also states the choices made where the
paper is silent (network shape, preprocessing, head outputs, emulated
rounding).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import Dict, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "_build", "liboracle.so")

#: sigma(TAU) == 0.3: detection threshold on the logit
TAU = math.log(0.3 / 0.7)

GCC_FLAGS = ["-O3", "-march=x86-64-v3", "-ffp-contract=off", "-fno-fast-math",
             "-fopenmp", "-fPIC", "-shared", "-std=c99"]


def build(force: bool = False) -> str:
    """Compile ``oracle.c`` into ``oracle/_build/liboracle.so`` (gcc, no fast-math,
    no FMA contraction, so every operation rounds as written)."""
    os.makedirs(os.path.dirname(_LIB), exist_ok=True)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", *GCC_FLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _L():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        d, i, l = ctypes.c_double, ctypes.c_int, ctypes.c_long
        P = ctypes.c_void_p
        _lib.or_round_bf16.restype = d
        _lib.or_round_bf16.argtypes = [d]
        _lib.or_round_e4m3.restype = d
        _lib.or_round_e4m3.argtypes = [d]
        _lib.or_fp8_group_exp.restype = i
        _lib.or_fp8_group_exp.argtypes = [d]
        _lib.or_store_fp8_groups.argtypes = [P, i, l]
        _lib.or_quant_weights_fp8.argtypes = [P, i, l]
        _lib.or_split_bf16.argtypes = [P, P, l]
        _lib.or_dense_maps.restype = i
        _lib.or_dense_maps.argtypes = [P, i, i, d, d, d, P, i, i, i, i, P, i, i, P]
        _lib.or_preprocess.argtypes = [P, l, d, d, d, P]
        _lib.or_conv3x3.argtypes = [P, i, i, i, P, P, i, i, P]
        _lib.or_net_maps.restype = i
        _lib.or_net_maps.argtypes = [P, i, i, d, d, d, P, i, i, P, i, i, P]
        _lib.or_preprocess_maps.argtypes = [P, l, P, P, d, P]
        _lib.or_net_maps_cam.restype = i
        _lib.or_net_maps_cam.argtypes = [P, i, i, P, P, d, P, i, i, P, i, i, P]
        _lib.or_detect.argtypes = [P, i, i, d, P]
        _lib.or_gate_pool.argtypes = [P, i, i, i, P]
        _lib.or_gate_forward.argtypes = [P, i, i, i, P, P]
        _lib.or_bce.restype = d
        _lib.or_bce.argtypes = [P, P, i, P]
        _lib.or_gate_backward.argtypes = [P, i, i, i, P, P, P]
        _lib.or_adam_step.argtypes = [P, P, P, P, i, i, d, d, d, d]
    return _lib


def _p(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


# ----------------------------------------------------------------- rounding
def round_bf16(v: np.ndarray) -> np.ndarray:
    v = np.asarray(v, np.float64)
    f = np.vectorize(_L().or_round_bf16, otypes=[np.float64])
    return f(v)


def round_e4m3(v: np.ndarray) -> np.ndarray:
    v = np.asarray(v, np.float64)
    f = np.vectorize(_L().or_round_e4m3, otypes=[np.float64])
    return f(v)


def fp8_group_exp(amax: float) -> int:
    """Exponent k of the FP8 group scale 2^k (smallest with amax <= 448 2^k,
    at least -126)."""
    return int(_L().or_fp8_group_exp(float(amax)))


def store_fp8_groups(a: np.ndarray) -> np.ndarray:
    """FP8 storage of a planar [C][...] tensor: per pixel, groups of 32
    channels share one power-of-two scale."""
    out = np.ascontiguousarray(a, np.float64).copy()
    C = out.shape[0]
    _L().or_store_fp8_groups(_p(out), C, out.size // C)
    return out


def split_bf16(v: np.ndarray):
    """(hi, lo) BF16 halves of the FP32 values v: hi = bf16(v), lo = bf16(v - hi)."""
    hi = np.ascontiguousarray(v, np.float64).copy()
    lo = np.empty_like(hi)
    _L().or_split_bf16(_p(hi), _p(lo), hi.size)
    return hi, lo


def quant_weights_fp8(W: np.ndarray) -> np.ndarray:
    """FP8 e4m3 quantisation of a convolution weight tensor [cout][...] with one
    scale per output channel, max|W[o]| / 448 (FP32); returns the dequantised
    FP64 values the FP8 emulation multiplies with."""
    out = np.ascontiguousarray(W, np.float64).copy()
    cout = out.shape[0]
    _L().or_quant_weights_fp8(_p(out), cout, out.size // cout)
    return out


# ----------------------------------------------------------- preprocessing
def _is_map(v) -> bool:
    return np.ndim(v) > 0


def _camera_maps(gain, offset, shape):
    """Per-pixel (sCMOS) gain and offset maps of `shape` as FP64 arrays (a
    scalar beside a map is broadcast)."""
    g = np.ascontiguousarray(np.broadcast_to(np.asarray(gain, np.float64), shape), np.float64)
    o = np.ascontiguousarray(np.broadcast_to(np.asarray(offset, np.float64), shape), np.float64)
    return g, o


def preprocess(frames: np.ndarray, gain, offset, in_scale: float) -> np.ndarray:
    """x = (ADU - offset) * gain * in_scale; gain and offset are scalars or
    per-pixel maps of one frame's shape (sCMOS)."""
    F = np.ascontiguousarray(frames, np.uint16)
    x = np.empty(F.shape, np.float64)
    if _is_map(gain) or _is_map(offset):
        g, o = _camera_maps(gain, offset, F.shape[-2:])
        for k in range(F.size // g.size):
            Fk = np.ascontiguousarray(F.reshape(-1, *g.shape)[k])
            xk = np.empty(g.shape, np.float64)
            _L().or_preprocess_maps(_p(Fk), g.size, _p(g), _p(o), in_scale, _p(xk))
            x.reshape(-1, *g.shape)[k] = xk
        return x
    _L().or_preprocess(_p(F), F.size, gain, offset, in_scale, _p(x))
    return x


# ------------------------------------------------------------- convolution
def conv3x3(x: np.ndarray, W: np.ndarray, b: Optional[np.ndarray], d: int) -> np.ndarray:
    """One 3x3 convolution with dilation ``d``: x [cin][h][w] -> [cout][h][w]."""
    x = np.ascontiguousarray(x, np.float64)
    W = np.ascontiguousarray(W, np.float64)
    cin, h, w = x.shape
    cout = W.shape[0]
    assert W.shape == (cout, cin, 3, 3)
    out = np.empty((cout, h, w), np.float64)
    bb = None if b is None else np.ascontiguousarray(b, np.float64)
    _L().or_conv3x3(_p(x), cin, h, w, _p(W), None if bb is None else _p(bb), cout, int(d), _p(out))
    return out


# ------------------------------------------------------------- the network
QUANT = {"fp32": 0, "fp64": 0, "exact": 0, "bf16": 1, "fp8": 2, "bf16x3": 3}


def _flat(spec, weights: Dict[str, np.ndarray]) -> np.ndarray:
    from smlm_synth import flat_weights
    return np.ascontiguousarray(flat_weights(spec, weights), np.float32)


def net_maps(frame: np.ndarray, spec, weights: Dict[str, np.ndarray], gain=0.5,
             offset=100.0, quant: str = "exact") -> np.ndarray:
    """Maps [nh][h][w] of one uint16 frame, FP64: logit, dx, dy, dz, photons
    (nh = 5), then the raw uncertainties of x, y, z, photons and the raw
    background (nh = 10).  gain and offset are scalars or per-pixel [h][w]
    maps (sCMOS)."""
    F = np.ascontiguousarray(frame, np.uint16)
    h, w = F.shape
    params = _flat(spec, weights)
    dil = np.asarray(spec.dilations, np.int32)
    nh = spec.head_outputs
    maps = np.empty((nh, h, w), np.float64)
    if hasattr(spec, "growth"):
        # the dense-connection network (FP64 only, scalar camera model)
        if quant != "exact" and QUANT[quant] != 0:
            raise ValueError("the dense-connection network has no emulation modes")
        if _is_map(gain) or _is_map(offset):
            raise ValueError("camera maps are not supported for the dense-connection network")
        rc = _L().or_dense_maps(_p(F), h, w, gain, offset, spec.in_scale, _p(params), spec.C, len(spec.dilations),
                                spec.layers, spec.growth, _p(dil), getattr(spec, "unet", 0), nh, _p(maps))
        if rc != 0:
            raise RuntimeError("oracle net failed")
        return maps
    if _is_map(gain) or _is_map(offset):
        g, o = _camera_maps(gain, offset, (h, w))
        rc = _L().or_net_maps_cam(_p(F), h, w, _p(g), _p(o), spec.in_scale, _p(params), spec.C,
                                  len(spec.dilations), _p(dil), QUANT[quant], nh, _p(maps))
    else:
        rc = _L().or_net_maps(_p(F), h, w, gain, offset, spec.in_scale, _p(params), spec.C,
                              len(spec.dilations), _p(dil), QUANT[quant], nh, _p(maps))
    if rc != 0:
        raise RuntimeError("oracle net failed")
    return maps


def net_maps_batch(frames: np.ndarray, spec, weights, gain=0.5, offset=100.0, quant="exact"):
    return np.stack([net_maps(f, spec, weights, gain, offset, quant) for f in frames])


def unet_reach(spec) -> int:
    """How far (pixels, per axis) the two-stage U-Net's output at a pixel
    reaches into its input a0, found by following the stage's row dependencies
    for every phase of the pixel modulo 4 (0 without a U-Net)."""
    if not getattr(spec, "unet", 0):
        return 0
    reach = 0
    for y in range(4, 8):
        rows = set()
        c0 = range(y - 1, y + 2)                              # final 3x3 conv at level 0
        rows |= set(c0)                                       # its skip input a0
        u1 = {r // 2 for r in c0}                             # up(u1) -> u1 rows
        c1 = {q for r in u1 for q in range(r - 1, r + 2)}     # u1's 3x3 conv at level 1
        d1 = set(c1) | {q for r in {r // 2 for r in c1} for q in range(2 * (r - 1), 2 * (r + 1) + 2)}
        # d1 rows come from d1 (skip) and from d2 = conv(pool(d1)); d1 = conv(pool(a0))
        for r in d1:
            rows |= set(range(2 * (r - 1), 2 * (r + 1) + 2))
        reach = max(reach, max(abs(r - y) for r in rows))
    return reach


def net_maps_window(frame: np.ndarray, spec, weights, y0: int, x0: int, hh: int, ww: int,
                    gain=0.5, offset=100.0, quant="exact", margin: Optional[int] = None) -> np.ndarray:
    """Exact maps of the output window [y0, y0+hh) x [x0, x0+ww) of a large frame.

    The net reads at most ``R = 1 + 2 * sum(dilations)`` pixels away (two
    convolutions per residual block; ``1 + L * sum(dilations)`` for the
    dense-connection network, L convolutions per block), so running it on the
    frame cropped to the window plus an R-pixel margin gives exact values
    inside the window (the crop edge coincides with the frame edge where the
    margin is clipped, and is at least R away elsewhere)."""
    H, W = frame.shape
    per_block = spec.layers if hasattr(spec, "growth") else 2
    R = 1 + per_block * sum(spec.dilations) + unet_reach(spec) if margin is None else margin
    # a U-Net's pooling windows start at even pixels of every level: the crop
    # starts at a multiple of 2^levels so they fall where they fall in the frame
    al = 2 ** getattr(spec, "unet", 0)
    cy0, cx0 = max(0, y0 - R) // al * al, max(0, x0 - R) // al * al
    cy1, cx1 = min(H, y0 + hh + R), min(W, x0 + ww + R)
    crop = frame[cy0:cy1, cx0:cx1]
    if _is_map(gain):
        gain = np.asarray(gain)[cy0:cy1, cx0:cx1]
    if _is_map(offset):
        offset = np.asarray(offset)[cy0:cy1, cx0:cx1]
    m = net_maps(crop, spec, weights, gain, offset, quant)
    return m[:, y0 - cy0:y0 - cy0 + hh, x0 - cx0:x0 - cx0 + ww]


# --------------------------------------------------------------- detection
def detect(logit: np.ndarray, tau: float = TAU) -> np.ndarray:
    """bool [h][w]: logit > tau and a strict winner of its 3x3 neighbourhood in
    the order (value, then smaller raster index)."""
    L = np.ascontiguousarray(logit, np.float64)
    h, w = L.shape
    det = np.empty((h, w), np.uint8)
    _L().or_detect(_p(L), h, w, float(tau), _p(det))
    return det.astype(bool)


EMITTER_DTYPE = np.dtype([("frame", "<i4"), ("row", "<i4"), ("col", "<i4"), ("x", "<f8"),
                          ("y", "<f8"), ("z", "<f8"), ("photons", "<f8"), ("prob", "<f8")])


def records(maps: np.ndarray, det: np.ndarray, spec, frame: int = 0) -> np.ndarray:
    """Emitter records of one frame in raster order: x = col + 0.5 + dx,
    y = row + 0.5 + dy (pixel centres), z = dz * z_scale, photons = ph * ph_scale,
    prob = 1 / (1 + exp(-logit))."""
    rows, cols = np.nonzero(det)            # row-major order == raster order
    out = np.empty(rows.size, EMITTER_DTYPE)
    out["frame"] = frame
    out["row"] = rows
    out["col"] = cols
    out["x"] = cols + 0.5 + maps[1, rows, cols]
    out["y"] = rows + 0.5 + maps[2, rows, cols]
    out["z"] = maps[3, rows, cols] * spec.z_scale
    out["photons"] = maps[4, rows, cols] * spec.ph_scale
    out["prob"] = 1.0 / (1.0 + np.exp(-maps[0, rows, cols]))
    return out


UNCERTAINTY_DTYPE = np.dtype([("sigma_x", "<f8"), ("sigma_y", "<f8"), ("sigma_z", "<f8"),
                               ("sigma_photons", "<f8"), ("background", "<f8")])


def softplus(u):
    """log(1 + e^u), in the form that neither overflows nor loses small values:
    max(u, 0) + log1p(e^-|u|)."""
    u = np.asarray(u, np.float64)
    return np.maximum(u, 0.0) + np.log1p(np.exp(-np.abs(u)))


# The least standard deviation the uncertainty planes express (units of the
# head: px, z_scale, ph_scale).  Without it the training loss's pixel mixture
# has no bounded likelihood: a target dimension that never varies (z in 2D
# data) lets sigma go to zero.
SIGMA_FLOOR = 0.01


def sigma_of(u):
    """A standard deviation from its raw plane: softplus(u) + SIGMA_FLOOR."""
    return softplus(u) + SIGMA_FLOOR


def uncertainties(maps: np.ndarray, det: np.ndarray, spec) -> np.ndarray:
    """Uncertainties of one frame's detections (raster order) from a 10-plane
    map: each sigma is sigma_of(raw plane) (positive by construction) times its
    unit -- sigma_x, sigma_y in px, sigma_z * z_scale (nm), sigma_photons *
    ph_scale; the background is softplus(raw) / in_scale (photons per pixel,
    the units the input scaling divides out)."""
    assert maps.shape[0] == 10, "the uncertainty head has 10 planes"
    rows, cols = np.nonzero(det)
    out = np.empty(rows.size, UNCERTAINTY_DTYPE)
    sp = [sigma_of(maps[5 + q, rows, cols]) for q in range(4)] + [softplus(maps[9, rows, cols])]
    out["sigma_x"] = sp[0]
    out["sigma_y"] = sp[1]
    out["sigma_z"] = sp[2] * spec.z_scale
    out["sigma_photons"] = sp[3] * spec.ph_scale
    out["background"] = sp[4] / spec.in_scale
    return out


def sigma_filter(maps: np.ndarray, det: np.ndarray, max_sigma_px: float) -> np.ndarray:
    """Uncertainty-aware post-processing of a 10-plane map: a detection is kept
    only if sigma_x = sigma_of(plane 5) and sigma_y = sigma_of(plane 6) are both
    <= max_sigma_px.  Applied after the local-maximum test, so a dropped
    maximum does not promote a neighbour."""
    assert maps.shape[0] == 10, "the uncertainty filter needs the 10-output head"
    return det & (sigma_of(maps[5]) <= max_sigma_px) & (sigma_of(maps[6]) <= max_sigma_px)


def localize(frames: np.ndarray, spec, weights, gain=0.5, offset=100.0, threshold=0.3,
             quant="exact", return_maps=False, with_uncertainty=False, max_sigma_px=0.0):
    """Whole path: frames -> maps -> detections -> records (frame, row, col order).
    gain and offset are scalars or per-pixel [h][w] maps shared by all frames.
    with_uncertainty (10-output heads): also the records' uncertainties, in
    the same order; returns (records, uncertainties[, maps]).  max_sigma_px > 0
    (10-output heads): drop detections whose sigma_x or sigma_y exceeds it."""
    tau = math.log(threshold / (1.0 - threshold))
    recs, uncs, allmaps = [], [], []
    for f, F in enumerate(frames):
        m = net_maps(F, spec, weights, gain, offset, quant)
        det = detect(m[0], tau)
        if max_sigma_px > 0:
            det = sigma_filter(m, det, max_sigma_px)
        recs.append(records(m, det, spec, f))
        if with_uncertainty:
            uncs.append(uncertainties(m, det, spec))
        if return_maps:
            allmaps.append(m)
    r = np.concatenate(recs) if recs else np.empty(0, EMITTER_DTYPE)
    out = [r]
    if with_uncertainty:
        out.append(np.concatenate(uncs) if uncs else np.empty(0, UNCERTAINTY_DTYPE))
    if return_maps:
        out.append(np.stack(allmaps))
    return out[0] if len(out) == 1 else tuple(out)


# -------------------------------------------------------------------- gate
GATE_NPARAM = 673


def gate_pool(x_tile: np.ndarray, pool: int = 4) -> np.ndarray:
    x = np.ascontiguousarray(x_tile, np.float64)
    th, tw = x.shape
    p = np.empty((th // pool, tw // pool), np.float64)
    _L().or_gate_pool(_p(x), th, tw, pool, _p(p))
    return p


def gate_forward(pooled: np.ndarray, theta: np.ndarray) -> np.ndarray:
    P = np.ascontiguousarray(pooled, np.float64)
    th = np.ascontiguousarray(theta, np.float64)
    assert th.size == GATE_NPARAM
    n, ph, pw = P.shape
    g = np.empty(n, np.float64)
    _L().or_gate_forward(_p(P), n, ph, pw, _p(th), _p(g))
    return g


def bce(g: np.ndarray, y: np.ndarray):
    g = np.ascontiguousarray(g, np.float64)
    y = np.ascontiguousarray(y, np.float64)
    dg = np.empty_like(g)
    L = _L().or_bce(_p(g), _p(y), g.size, _p(dg))
    return L, dg


def gate_backward(pooled: np.ndarray, theta: np.ndarray, dg: np.ndarray) -> np.ndarray:
    P = np.ascontiguousarray(pooled, np.float64)
    th = np.ascontiguousarray(theta, np.float64)
    dg = np.ascontiguousarray(dg, np.float64)
    n, ph, pw = P.shape
    grad = np.empty(GATE_NPARAM, np.float64)
    _L().or_gate_backward(_p(P), n, ph, pw, _p(th), _p(dg), _p(grad))
    return grad


def adam_step(theta, m, v, grad, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """In-place Adam update of float64 arrays theta, m, v."""
    for a in (theta, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = np.ascontiguousarray(grad, np.float64)
    _L().or_adam_step(_p(theta), _p(m), _p(v), _p(g), theta.size, int(t), lr, b1, b2, eps)
