"""Comparison helpers for GPU-vs-oracle parity (shared by the tests, smoke and bench).

Readings used:
* maps: |gpu - oracle| <= tol * (|oracle| + rms of that map over the frame),
  a relative error that stays defined where a map crosses zero;
* emitter sets: identical except pixels the FP64 oracle puts within 1e-3 of the
  probability threshold, or whose logit ties a neighbour's to 1e-4 relative
  (there the FP32 rounding decides the local maximum); such pixels are exempt
  and counted.
"""
from __future__ import annotations

import math

import numpy as np


def map_rel_err(got: np.ndarray, ref: np.ndarray) -> np.ndarray:
    """Max relative error per map plane; arrays [n][5][h][w] (or [5][h][w])."""
    g = np.asarray(got, np.float64)
    r = np.asarray(ref, np.float64)
    if g.ndim == 3:
        g, r = g[None], r[None]
    out = np.zeros(r.shape[1])
    for c in range(r.shape[1]):
        rms = np.sqrt(np.mean(r[:, c] ** 2)) or 1.0
        out[c] = np.max(np.abs(g[:, c] - r[:, c]) / (np.abs(r[:, c]) + rms))
    return out


def exempt_mask(logit: np.ndarray, threshold: float = 0.3, band: float = 1e-3, tie: float = 1e-4) -> np.ndarray:
    """Pixels whose detection decision FP32 rounding may legitimately flip."""
    L = np.asarray(logit, np.float64)
    p = 1.0 / (1.0 + np.exp(-L))
    ex = np.abs(p - threshold) <= band
    h, w = L.shape
    pad = np.pad(L, 1, constant_values=np.nan)
    for di in (-1, 0, 1):
        for dj in (-1, 0, 1):
            if di == 0 and dj == 0:
                continue
            nb = pad[1 + di:1 + di + h, 1 + dj:1 + dj + w]
            with np.errstate(invalid="ignore"):
                ex |= np.abs(L - nb) <= tie * (1.0 + np.abs(L))
    return ex


def compare_emitters(got, ref, ref_maps: np.ndarray, threshold: float = 0.3):
    """got: records with fields frame,row,col,(x_px|x),(y_px|y),...; ref: oracle records;
    ref_maps: [n][5][h][w] oracle maps.  Returns a summary dict."""
    gk = {(int(a), int(b), int(c)): i for i, (a, b, c) in enumerate(zip(got["frame"], got["row"], got["col"]))}
    rk = {(int(a), int(b), int(c)): i for i, (a, b, c) in enumerate(zip(ref["frame"], ref["row"], ref["col"]))}
    ex = [exempt_mask(ref_maps[f, 0], threshold) for f in range(ref_maps.shape[0])]
    only_g = [k for k in gk if k not in rk]
    only_r = [k for k in rk if k not in gk]
    bad = [k for k in only_g + only_r if not ex[k[0]][k[1], k[2]]]
    both = [k for k in gk if k in rk]
    gx = got["x_px"] if "x_px" in got.dtype.names else got["x"]
    gy = got["y_px"] if "y_px" in got.dtype.names else got["y"]
    dx = np.array([gx[gk[k]] - ref["x"][rk[k]] for k in both]) if both else np.zeros(0)
    dy = np.array([gy[gk[k]] - ref["y"][rk[k]] for k in both]) if both else np.zeros(0)
    gz = got["z_nm"] if "z_nm" in got.dtype.names else got["z"]
    dz = np.array([gz[gk[k]] - ref["z"][rk[k]] for k in both]) if both else np.zeros(0)
    order_ok = list(zip(got["frame"], got["row"], got["col"])) == sorted(zip(got["frame"], got["row"], got["col"]))
    n_ref = len(rk)
    return {
        "n_got": len(gk), "n_ref": n_ref, "matched": len(both),
        "only_gpu": len(only_g), "only_oracle": len(only_r), "non_exempt_mismatch": len(bad),
        "bad": bad[:10], "order_ok": order_ok,
        "recall": len(both) / n_ref if n_ref else 1.0,
        "precision": len(both) / len(gk) if gk else 1.0,
        "rms_dx_px": float(np.sqrt(np.mean(dx ** 2))) if dx.size else 0.0,
        "rms_dy_px": float(np.sqrt(np.mean(dy ** 2))) if dy.size else 0.0,
        "rms_dz_nm": float(np.sqrt(np.mean(dz ** 2))) if dz.size else 0.0,
        "max_dxy_px": float(max(np.abs(dx).max(initial=0), np.abs(dy).max(initial=0))),
    }


def logit_tau(threshold: float = 0.3) -> float:
    return math.log(threshold / (1.0 - threshold))


def match_by_distance(got, ref, radius: float = 1.0):
    """One-to-one matching of emitters by position within the same frame:
    pairs are taken greedily in order of increasing distance, up to ``radius``
    pixels.  Used for the reduced-precision and gated forms, whose local
    maximum may move to an adjacent pixel.  Returns recall, precision and the
    RMS coordinate differences over matched pairs."""
    from scipy.spatial import cKDTree
    gx = np.asarray(got["x_px"] if "x_px" in got.dtype.names else got["x"], np.float64)
    gy = np.asarray(got["y_px"] if "y_px" in got.dtype.names else got["y"], np.float64)
    gz = np.asarray(got["z_nm"] if "z_nm" in got.dtype.names else got["z"], np.float64)
    rx, ry, rz = (np.asarray(ref[k], np.float64) for k in ("x", "y", "z"))
    pairs = []
    for f in np.union1d(np.unique(got["frame"]), np.unique(ref["frame"])):
        gi = np.flatnonzero(got["frame"] == f)
        ri = np.flatnonzero(ref["frame"] == f)
        if gi.size == 0 or ri.size == 0:
            continue
        tree = cKDTree(np.c_[rx[ri], ry[ri]])
        cand = tree.query_ball_point(np.c_[gx[gi], gy[gi]], r=radius)
        edges = [(np.hypot(gx[g] - rx[ri[r]], gy[g] - ry[ri[r]]), g, ri[r]) for g, rs in zip(gi, cand) for r in rs]
        edges.sort()
        used_g, used_r = set(), set()
        for d, g, r in edges:
            if g in used_g or r in used_r:
                continue
            used_g.add(g)
            used_r.add(r)
            pairs.append((g, r))
    m = len(pairs)
    if m:
        gi = np.array([p[0] for p in pairs])
        ri = np.array([p[1] for p in pairs])
        dx, dy, dz = gx[gi] - rx[ri], gy[gi] - ry[ri], gz[gi] - rz[ri]
    else:
        dx = dy = dz = np.zeros(0)
    return {"matched": m, "n_got": len(got), "n_ref": len(ref),
            "recall": m / len(ref) if len(ref) else 1.0, "precision": m / len(got) if len(got) else 1.0,
            "rms_dx_px": float(np.sqrt(np.mean(dx ** 2))) if m else 0.0,
            "rms_dy_px": float(np.sqrt(np.mean(dy ** 2))) if m else 0.0,
            "rms_dz_nm": float(np.sqrt(np.mean(dz ** 2))) if m else 0.0}


def record_field_errors(got, ref, ref_maps, spec, keys=None):
    """Worst error of each record field over the emitters both lists hold,
    each divided by the bound the FP32 map tolerance (1e-4 of |value| + the
    map's rms) implies for it; a value <= 1 is within tolerance.

    x, y: 1e-3 px (the offsets' 1e-4 bound plus FP32 rounding of
    col + 0.5 + dx at columns up to 2^12); z and photons: 1e-4 (|dz| + rms dz)
    times z_scale, likewise ph_scale; prob: the logit bound times the
    sigmoid's slope (at most 1/4) plus 1e-6.  ``ref_maps`` is [n][planes][h][w]
    for the frames the records index; ``keys`` restricts the comparison."""
    gk = {(int(a), int(b), int(c)): i for i, (a, b, c) in enumerate(zip(got["frame"], got["row"], got["col"]))}
    rk = {(int(a), int(b), int(c)): i for i, (a, b, c) in enumerate(zip(ref["frame"], ref["row"], ref["col"]))}
    both = [k for k in gk if k in rk and (keys is None or k in keys)]
    out = {"n": len(both), "x": 0.0, "y": 0.0, "z": 0.0, "photons": 0.0, "prob": 0.0}
    if not both:
        return out
    gi = np.array([gk[k] for k in both])
    ri = np.array([rk[k] for k in both])
    fr = np.array([k[0] for k in both])
    rms = {q: np.array([np.sqrt(np.mean(np.asarray(ref_maps[f, q], np.float64) ** 2)) for f in range(ref_maps.shape[0])])
           for q in (0, 3, 4)}
    gx = got["x_px"] if "x_px" in got.dtype.names else got["x"]
    gy = got["y_px"] if "y_px" in got.dtype.names else got["y"]
    gz = got["z_nm"] if "z_nm" in got.dtype.names else got["z"]
    out["x"] = float(np.max(np.abs(gx[gi] - ref["x"][ri])) / 1e-3)
    out["y"] = float(np.max(np.abs(gy[gi] - ref["y"][ri])) / 1e-3)
    zb = 1e-4 * (np.abs(ref["z"][ri]) + rms[3][fr] * spec.z_scale) + 1e-6
    out["z"] = float(np.max(np.abs(gz[gi] - ref["z"][ri]) / zb))
    pb = 1e-4 * (np.abs(ref["photons"][ri]) + rms[4][fr] * spec.ph_scale) + 1e-6
    out["photons"] = float(np.max(np.abs(got["photons"][gi] - ref["photons"][ri]) / pb))
    lg = np.array([ref_maps[k[0], 0, k[1], k[2]] for k in both], np.float64)   # the oracle's logits
    qb = 0.25 * 1e-4 * (np.abs(lg) + rms[0][fr]) + 1e-6
    out["prob"] = float(np.max(np.abs(got["prob"][gi] - ref["prob"][ri]) / qb))
    return out
