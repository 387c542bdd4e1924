"""Reader of tests/golden/tiny_oracle_records.txt (written by
tests/golden/make_golden.py from the oracle alone)."""
import os

import numpy as np

PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "tiny_oracle_records.txt")
FIELDS = [("frame", "<i4"), ("row", "<i4"), ("col", "<i4"), ("x", "<f8"), ("y", "<f8"), ("z", "<f8"),
          ("photons", "<f8"), ("prob", "<f8"), ("logit", "<f8")]


def load():
    """(records, set of near-decision (frame, row, col), per-frame counts)."""
    recs, near, counts = [], set(), None
    for line in open(PATH):
        if line.startswith("record "):
            v = line.split()[1:]
            recs.append(tuple(int(x) for x in v[:3]) + tuple(float(x) for x in v[3:]))
        elif line.startswith("near "):
            near.add(tuple(int(x) for x in line.split()[1:]))
        elif line.startswith("counts "):
            counts = [int(x) for x in line.split()[1:]]
    return np.array(recs, dtype=FIELDS), near, counts
