"""Writes tiny_oracle_records.txt: the FP64 oracle's emitter records for the
tiny workload (4 uint16 frames of 128 x 128, 2D Gaussian PSF, frame seed 1001;
net A, weight seed 1; gain 0.5, offset 100, threshold 0.3), which the tests
compare with the oracle (regression) and with the library (GPU parity).

It calls only the oracle and the seeded input generator.  Each record line
also carries the oracle's logit at that pixel, and the file lists the pixels
whose decision floating point may flip: the oracle puts their probability
within 1e-3 of the threshold, or a neighbour's logit within 1e-4 (relative)
of theirs.

Run from the repository root:  python tests/golden/make_golden.py
"""
import math
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))
import oracle  # noqa: E402
import smlm_synth as S  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tiny_oracle_records.txt")


def near_decision(logit):
    """Pixels whose detection a rounding can flip (same rule as the parity helpers)."""
    p = 1.0 / (1.0 + np.exp(-logit))
    near = np.abs(p - 0.3) <= 1e-3
    h, w = logit.shape
    pad = np.pad(logit, 1, constant_values=-np.inf)
    for di in (-1, 0, 1):
        for dj in (-1, 0, 1):
            if di == 0 and dj == 0:
                continue
            nb = pad[1 + di:1 + di + h, 1 + dj:1 + dj + w]
            near |= np.abs(nb - logit) <= 1e-4 * (1.0 + np.abs(logit))
    return near


def main():
    spec, w = S.make_net("A", 1)
    frames = S.render_frames(4, 128, 128, "tiny", 1001)
    rec, maps = oracle.localize(frames, spec, w, return_maps=True)
    lines = ["# FP64 oracle records, tiny workload: 4 x 128 x 128 frames (seed 1001), net A (seed 1),",
             "# gain 0.5, offset 100, threshold 0.3 (logit > ln(0.3/0.7)); written by make_golden.py",
             "# record: frame row col x_px y_px z_nm photons prob logit"]
    for r in rec:
        lg = maps[r["frame"], 0, r["row"], r["col"]]
        lines.append(f"record {r['frame']} {r['row']} {r['col']} {r['x']:.12g} {r['y']:.12g} {r['z']:.12g} "
                     f"{r['photons']:.12g} {r['prob']:.12g} {lg:.12g}")
    for f in range(len(frames)):
        ys, xs = np.nonzero(near_decision(maps[f, 0]))
        for y, x in zip(ys.tolist(), xs.tolist()):
            lines.append(f"near {f} {y} {x}")
    lines.append(f"counts {' '.join(str(int(np.sum(rec['frame'] == f))) for f in range(len(frames)))}")
    open(OUT, "w").write("\n".join(lines) + "\n")
    print(f"wrote {len(rec)} records to {OUT}")


if __name__ == "__main__":
    main()
