"""Host logic of the gate threshold (CPU): the threshold chosen for a recall
target gives up only the lowest-scored positives, by count or by weight."""
import numpy as np
import pytest

GT = pytest.importorskip("paper_2410_02314_amd.gate_train")


def kept(scores, t):
    return scores > t


def test_unit_weights_give_up_floor_fraction():
    r = np.random.default_rng(0)
    s = r.standard_normal(1000)
    pos = r.random(1000) < 0.4
    for target in (1.0, 0.995, 0.9, 0.5):
        t = GT.threshold_for_recall(s, pos, target)
        lost = np.count_nonzero(pos & ~kept(s, t))
        assert lost == int(np.floor((1 - target) * pos.sum() + 1e-9))
        assert np.all(s[pos & ~kept(s, t)] < np.min(s[pos & kept(s, t)]))


def test_weighted_recall_gives_up_light_positives():
    # three heavy positives and many light ones: 99 % of the weight can be kept
    # while giving up every light positive below the heavy ones
    s = np.array([0.1, 0.2, 0.3, 0.4, 5.0, 6.0, 7.0, -1.0])
    pos = np.array([True, True, True, True, True, True, True, False])
    w = np.array([1, 1, 1, 1, 300, 300, 300, 0], float)
    t = GT.threshold_for_recall(s, pos, 0.99, w)
    k = kept(s, t)
    assert not k[:4].any() and k[4:7].all()
    assert w[pos & k].sum() >= 0.99 * w[pos].sum()
    # unit weights at the same target may give up none of the seven
    t1 = GT.threshold_for_recall(s, pos, 0.99)
    assert kept(s, t1)[pos].all()


def test_no_positives_keeps_nothing_above_max():
    s = np.array([0.5, 1.5])
    t = GT.threshold_for_recall(s, np.zeros(2, bool), 0.995)
    assert not kept(s, t).any()


def test_tile_counts_and_labels():
    rec = np.zeros(4, dtype=[("frame", "<i4"), ("row", "<i4"), ("col", "<i4")])
    rec["frame"] = [0, 0, 1, 1]
    rec["row"] = [0, 10, 300, 511]
    rec["col"] = [0, 260, 5, 511]
    c = GT.tile_counts(rec, 2, 512, 512)
    assert list(c) == [1, 1, 0, 0, 0, 0, 1, 1]
    assert list(GT.tile_labels(rec, 2, 512, 512)) == [1, 1, 0, 0, 0, 0, 1, 1]
