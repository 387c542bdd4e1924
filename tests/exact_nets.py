"""Integer-valued networks on which the reduced-precision forms are exact
arithmetic, so the GPU's BF16 and FP8 results can be held to the oracle's
emulation bit for bit.

With gain 1, in_scale 1 and integer frames the preprocessed input is an
integer.  Every weight and bias below is an integer (times a power of two per
output channel for FP8), so every product and every partial sum is an integer
as long as it stays below 2^24: FP32 accumulation in any order, FP64
accumulation and the MFMA all give the same value.  Rounding therefore happens
only where the form stores a value:

* BF16 keeps 8 significant bits, so stored integers above 256 round (to an
  integer, ties to even);
* FP8 e4m3 keeps 4 significant bits; with the group scale a power of two, a
  stored integer rounds to an integer again.

FP8 weight scales: the FP8 form scales output channel o's weights by
max|W[o]| / 448.  Here channel o's weights are {-1, 0, 1} * 2^j[o] (j[o] in
{0, 1}) plus one entry 7 * 2^j[o], so max|W[o]| = 1.75 * 2^(j[o] + 2) and the
scale 2^(j[o] - 6) is exact; the quantised weights equal the weights.  The
7 * 2^j entry reads a dead input channel (always zero: its stem and conv rows
are zero), so it sets the scale without amplifying the activations.  j[o]
differs between channels, so a scale applied to the wrong output channel
changes the result.
"""
from __future__ import annotations

import numpy as np

import oracle
import smlm_synth as S


def _base(C: int, dil, tag: str) -> S.NetSpec:
    return S.NetSpec(f"{tag}{C}", C, tuple(dil), in_scale=1.0)


def bf16_integer_net(C: int = 16, dil=(1, 2), seed: int = 15, nnz: float = 3.0):
    """Sparse small-integer weights (about ``nnz`` non-zero taps per output
    channel), integer biases."""
    spec = _base(C, dil, "int")
    r = np.random.default_rng(seed)
    w = {}
    for n, s in S.tensor_layout(spec):
        if n.endswith(("w1", "w2")):
            p = nnz / (9.0 * C)
            w[n] = (r.integers(-1, 3, size=s) * (r.random(s) < p)).astype(np.float32)
        elif n == "stem.w":
            w[n] = r.integers(0, 2, size=s).astype(np.float32)
        elif n == "head.w":
            w[n] = r.integers(-1, 2, size=s).astype(np.float32)
        else:
            w[n] = r.integers(-1, 2, size=s).astype(np.float32)
    return spec, w


def fp8_exact_net(C: int = 48, dil=(1, 2, 4, 8, 16), seed: int = 21, nnz: float = 3.0):
    """See the module docstring: exact FP8 weight scales 2^(j[o] - 6), one dead
    input channel (the last), integer biases."""
    spec = _base(C, dil, "f8x")
    r = np.random.default_rng(seed)
    D = C - 1
    w = {}
    for n, s in S.tensor_layout(spec):
        if n == "stem.w":
            a = r.integers(0, 2, size=s).astype(np.float64)
            a[D] = 0
        elif n.endswith(("w1", "w2")):
            j = r.integers(0, 2, size=C)
            a = (r.integers(-1, 2, size=s) * (r.random(s) < nnz / (9.0 * C))).astype(np.float64)
            a[:, D] = 0
            tap = r.integers(0, 9, size=C)
            sign = np.where(r.random(C) < 0.5, -1.0, 1.0)
            for o in range(C):
                a[o, D, tap[o] // 3, tap[o] % 3] = 7.0 * sign[o]
            a *= (2.0 ** j)[:, None, None, None]
            a[D] = 0
        elif n.endswith(("b1", "b2", "stem.b")):
            a = r.integers(-2, 1, size=s).astype(np.float64)
            a[D] = 0
        elif n == "head.w":
            a = r.integers(-1, 2, size=s).astype(np.float64)
        else:
            a = r.integers(-2, 3, size=s).astype(np.float64)
        w[n] = a.astype(np.float32)
    return spec, w


def integer_frames(n: int, h: int, wd: int, seed: int, top: int = 24) -> np.ndarray:
    """uint16 frames 100 + U{0, .., top - 1}: preprocessed (offset 100, gain 1,
    in_scale 1) to integers 0 .. top - 1."""
    r = np.random.default_rng(seed)
    return (100 + r.integers(0, top, size=(n, h, wd))).astype(np.uint16)


def max_intermediate(frame: np.ndarray, spec, w, include_head: bool = True) -> float:
    """Largest magnitude of any pre-activation sum of the exact (unquantised)
    network on one frame: stem, each block's two convolutions (the second
    with its residual), head.  Rounding to BF16 or e4m3 changes a stored value
    by at most 1/16 of it, so a bound well below 2^24 here keeps the
    quantised network's sums exact too."""
    x = (frame.astype(np.float64) - 100.0)[None]
    m = 0.0
    a = oracle.conv3x3(x, w["stem.w"].astype(np.float64), w["stem.b"].astype(np.float64), 1)
    m = max(m, np.abs(a).max())
    a = np.maximum(a, 0)
    for k, d in enumerate(spec.dilations):
        t = oracle.conv3x3(a, w[f"blk{k}.w1"].astype(np.float64), w[f"blk{k}.b1"].astype(np.float64), d)
        m = max(m, np.abs(t).max())
        t = np.maximum(t, 0)
        u = a + oracle.conv3x3(t, w[f"blk{k}.w2"].astype(np.float64), w[f"blk{k}.b2"].astype(np.float64), d)
        m = max(m, np.abs(u).max())
        a = np.maximum(u, 0)
    if not include_head:
        return float(m)
    hw = w["head.w"].astype(np.float64)
    maps = np.tensordot(hw, a, axes=(1, 0)) + w["head.b"].astype(np.float64)[:, None, None]
    return float(max(m, np.abs(maps).max()))
