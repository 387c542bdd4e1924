"""The stored oracle records of the tiny workload (tests/golden) against the
oracle as it stands: any change of the oracle's arithmetic that moves a
record shows here."""
import numpy as np

import oracle
import smlm_synth as S
from tests.golden_records import load


def test_oracle_reproduces_the_stored_records():
    gold, near, counts = load()
    spec, w = S.make_net("A", 1)
    frames = S.render_frames(4, 128, 128, "tiny", 1001)
    rec, maps = oracle.localize(frames, spec, w, return_maps=True)
    assert len(rec) == len(gold) == sum(counts)
    for f in ("frame", "row", "col"):
        assert np.array_equal(rec[f], gold[f])
    for f in ("x", "y", "z", "photons", "prob"):
        assert np.allclose(rec[f], gold[f], rtol=1e-10, atol=1e-12), f
    assert np.allclose(maps[gold["frame"], 0, gold["row"], gold["col"]], gold["logit"], rtol=1e-10, atol=1e-12)
    assert list(np.bincount(rec["frame"], minlength=4)) == counts
    assert all(0 <= f < 4 and 0 <= y < 128 and 0 <= x < 128 for f, y, x in near)
