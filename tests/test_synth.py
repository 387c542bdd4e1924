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


def test_scmos_camera_is_seeded_and_plausible():
    a, b = S.scmos_camera(64, 96, 7), S.scmos_camera(64, 96, 7)
    assert all(np.array_equal(getattr(a, k), getattr(b, k)) for k in ("gain", "offset", "read_sd"))
    c = S.scmos_camera(64, 96, 8)
    assert not np.array_equal(a.offset, c.offset)
    assert a.gain.dtype == np.float32 and a.gain.shape == (64, 96)
    assert np.all(a.gain > 0.5 * 0.79) and np.all(a.gain < 0.5 * 1.21) and abs(a.gain.mean() - 0.5) < 0.005
    assert abs(a.offset.mean() - 100.0) < 0.2 and 2.5 < a.offset.std() < 3.5
    assert np.all(a.read_sd > 0)


def test_constant_camera_renders_the_scalar_model():
    """A camera whose maps equal the model's scalars draws the same random
    numbers in the same order: the frames are identical."""
    h, w = 48, 80
    cam = S.Camera(np.full((h, w), 0.5, np.float32), np.full((h, w), 100.0, np.float32),
                   np.full((h, w), 1.5, np.float32))
    a = S.render_frames(2, h, w, "tiny", 5)
    b = S.render_frames(2, h, w, "tiny", 5, camera=cam)
    assert np.array_equal(a, b)


def test_camera_offset_shows_in_dark_frames():
    """Background only (no emitters): each pixel's mean ADU over many frames
    approaches offset + background / gain of that pixel."""
    import dataclasses
    h, w = 8, 12
    cam = S.scmos_camera(h, w, 3, offset_sd=20.0)
    dark = dataclasses.replace(S.CONFIG_MODELS["tiny"], density=(0.0, 0.0), background=(10.0, 10.0))
    fr = S.render_frames(400, h, w, dark, 9, camera=cam, workers=1).astype(np.float64)
    expect = cam.offset + 10.0 / cam.gain
    assert np.abs(fr.mean(axis=0) - expect).max() < 1.5
