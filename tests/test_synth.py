"""Host checks of the seeded frame generator's empty-tile layouts."""
import numpy as np
import pytest

import smlm_synth as S


def _components(occ):
    """Number of 4-connected components of True cells."""
    seen = np.zeros_like(occ, bool)
    n = 0
    for y, x in zip(*np.nonzero(occ)):
        if seen[y, x]:
            continue
        n += 1
        stack = [(y, x)]
        seen[y, x] = True
        while stack:
            a, b = stack.pop()
            for c, d in ((a + 1, b), (a - 1, b), (a, b + 1), (a, b - 1)):
                if 0 <= c < occ.shape[0] and 0 <= d < occ.shape[1] and occ[c, d] and not seen[c, d]:
                    seen[c, d] = True
                    stack.append((c, d))
    return n


@pytest.mark.parametrize("q", [0.3, 0.5, 0.7])
def test_cell_layout_empty_fraction_and_one_region(q):
    rng = np.random.default_rng(17)
    for _ in range(20):
        occ = S._occupancy(8, 8, q, "cell", rng)
        assert occ.sum() == round((1 - q) * 64)
        assert _components(occ) == 1


def test_iid_layout_fraction():
    rng = np.random.default_rng(18)
    occ = S._occupancy(256, 256, 0.4, "iid", rng)
    assert abs(1 - occ.mean() - 0.4) < 0.01


def test_unknown_layout_rejected():
    with pytest.raises(ValueError):
        S._occupancy(4, 4, 0.5, "stripes", np.random.default_rng(0))


@pytest.mark.parametrize("model", ["sparse", "sparse_cell"])
def test_emitters_only_in_occupied_tiles(model):
    fr, truth = S.render_frames(2, 512, 512, model, 77, with_truth=True, workers=1)
    for t in truth:
        occ = t["tile_occupied"]
        ty = (np.asarray(t["y"]) // 256).astype(int)
        tx = (np.asarray(t["x"]) // 256).astype(int)
        assert occ[ty, tx].all()
