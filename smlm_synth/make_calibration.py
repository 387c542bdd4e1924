"""Compute the head-calibration constants of the seeded random networks.

Writes ``smlm_synth/calibration.json``.  Only the FP64 oracle computes the
network outputs used here, so no stored input ever depends on the HIP path.

A randomly initialised network has no reason to put its logit threshold
between emitters and background.  For each (net, seed) this script keeps the
He-normal stem and blocks and replaces only the 1x1 head by a linear probe of
the final features, fitted on seeded calibration frames (background only, and
sparse emitters with known positions):

1. logit row: the Fisher/LDA direction Sigma_bg^-1 (mu_emitter - mu_bg),
   scaled to unit spread on background; its bias puts the largest background
   logit a quarter of the way from the background maximum towards the median
   emitter logit, below the detection threshold;
2. dx, dy, dz, photon rows: least-squares fits of the true sub-pixel offset,
   z / z_scale and photons / ph_scale at the pixel holding each emitter.

The final features are read through the head itself (five unit rows at a
time), so only the oracle's own network function is used.

Run:  python -m smlm_synth.make_calibration [net ...]
"""
from __future__ import annotations

import json
import math
import os

import numpy as np

import oracle
import smlm_synth as S

CAL_SEEDS = {"A": 1, "B": 2, "D": 3, "DU": 3}
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "calibration.json")


def _features(frame, spec, w):
    """Final feature maps [C][h][w] of the oracle network, read through the head."""
    C = spec.C
    feats = []
    for c0 in range(0, C, 5):
        ww = dict(w)
        hw = np.zeros((5, C), np.float32)
        for q in range(5):
            if c0 + q < C:
                hw[q, c0 + q] = 1.0
        ww["head.w"] = hw
        ww["head.b"] = np.zeros(5, np.float32)
        m = oracle.net_maps(frame, spec, ww)
        feats.extend(m[q] for q in range(5) if c0 + q < C)
    return np.stack(feats)


def calibrate(name: str, seed: int) -> dict:
    spec, w = S.make_net(name, seed, calibrated=False)
    base = S.CONFIG_MODELS["tiny"] if name == "A" else S.CONFIG_MODELS["full"]
    n = 320
    fbs, fes, tgt = [], [], [[], [], [], []]
    bgs = sorted(set(base.background))
    if bgs[0] != bgs[-1]:
        bgs = [bgs[0], 0.5 * (bgs[0] + bgs[-1]), bgs[-1]]
    for k, b in enumerate(bgs):
        bg = S.render_frames(1, n, n, S.replace(base, density=(0.0, 0.0), background=(b, b)),
                             9000 + 10 * seed + k)[0]
        fbs.append(_features(bg, spec, w).reshape(spec.C, -1).T)             # (pixels, C)
        em, tr = S.render_frames(1, n, n, S.replace(base, density=(0.3, 0.3), background=(b, b)),
                                 9100 + 10 * seed + k, with_truth=True)
        t = tr[0]
        ys = np.clip(np.floor(t["y"]).astype(int), 0, n - 1)
        xs = np.clip(np.floor(t["x"]).astype(int), 0, n - 1)
        fes.append(_features(em[0], spec, w)[:, ys, xs].T)                    # (emitters, C)
        tgt[0].append(t["x"] - (xs + 0.5))
        tgt[1].append(t["y"] - (ys + 0.5))
        tgt[2].append(t["z_nm"] / spec.z_scale)
        tgt[3].append(t["photons"] / spec.ph_scale)
    fb = np.concatenate(fbs)
    fe = np.concatenate(fes)
    targets = [np.concatenate(v) for v in tgt]
    xs = fe[:, 0]

    mu_b, mu_e = fb.mean(0), fe.mean(0)
    cov = np.cov(fb.T) + 1e-3 * np.eye(spec.C) * np.trace(np.cov(fb.T)) / spec.C
    wl = np.linalg.solve(cov, mu_e - mu_b)
    wl /= float(np.std(fb @ wl)) or 1.0
    em_sc = fe @ wl
    bg_max = float(np.max(fb @ wl))
    em_med = float(np.median(em_sc))
    gap = em_med - bg_max
    level = bg_max + (0.25 * gap if gap > 0 else 0.5)
    head_w = np.zeros((5, spec.C))
    head_b = np.zeros(5)
    head_w[0] = wl
    head_b[0] = S.TAU_LOGIT - level
    # least-squares rows for offsets / z / photons at the emitter pixels
    X = np.concatenate([fe, np.ones((fe.shape[0], 1))], axis=1)
    for q, y in enumerate(targets, start=1):
        coef, *_ = np.linalg.lstsq(X, y, rcond=None)
        head_w[q] = coef[:-1]
        head_b[q] = coef[-1]
    return {"head_w": head_w.astype(np.float32).tolist(), "head_b": head_b.astype(np.float32).tolist(),
            "stats": {"bg_max": bg_max, "em_median": em_med, "n_emitters": int(xs.size),
                      "em_above_bg_max": float(np.mean(em_sc > bg_max))}}


def main(argv=None):
    """Calibrate every (net, seed), or only the nets named on the command line
    (the other entries of the existing file are kept)."""
    import sys
    names = (argv if argv is not None else sys.argv[1:]) or list(CAL_SEEDS)
    table = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            table = json.load(f)
    for name in names:
        seed = CAL_SEEDS[name]
        table[f"{name}:{seed}"] = calibrate(name, seed)
        print(name, seed, json.dumps(table[f"{name}:{seed}"]["stats"]))
    with open(OUT, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
        f.write("\n")


if __name__ == "__main__":
    main()
