"""Pins of the oracle's per-pixel (sCMOS) camera maps, x = (ADU - offset[p]) *
gain[p] * in_scale, against the scalar path it generalises:

* constant maps give the scalar path's result bit for bit;
* per-pixel equivalence: gain k[p] * g and offset o[p] on frame F equal the
  scalar gain g and offset o_s on the frame F' = o_s + k[p] (F - o[p]) (an
  integer frame), so a transposed, shifted or swapped map fails;
* locality: changing the offset of one pixel changes the maps only within the
  network's receptive radius of that pixel, and there it does change them."""
import numpy as np
import pytest

import oracle
import smlm_synth as S


@pytest.fixture(scope="module")
def net():
    return S.make_net("A", 1)


def test_constant_maps_equal_scalar_path(net):
    spec, w = net
    F = S.render_frames(1, 40, 56, "tiny", 5)[0]
    a = oracle.net_maps(F, spec, w, 0.5, 100.0)
    b = oracle.net_maps(F, spec, w, np.full((40, 56), 0.5), np.full((40, 56), 100.0))
    assert np.array_equal(a, b)


def test_per_pixel_maps_equal_rescaled_frame(net):
    spec, w = net
    h, wd = 37, 52                                    # non-square: a transposed map cannot fit
    rng = np.random.default_rng(11)
    o_map = rng.integers(90, 111, size=(h, wd)).astype(np.float64)
    k = rng.integers(1, 4, size=(h, wd)).astype(np.float64)
    F = (o_map + rng.integers(0, 200, size=(h, wd))).astype(np.uint16)
    g, o_s = 0.5, 100.0
    Fp = o_s + k * (F.astype(np.float64) - o_map)
    assert Fp.min() >= 0 and Fp.max() < 65536
    Fp = Fp.astype(np.uint16)
    a = oracle.net_maps(F, spec, w, k * g, o_map)
    b = oracle.net_maps(Fp, spec, w, g, o_s)
    assert np.allclose(a, b, rtol=1e-12, atol=1e-12 * np.abs(b).max())
    # the preprocessed inputs agree exactly (powers of two and small integers)
    xa = oracle.preprocess(F, k * g, o_map, spec.in_scale)
    xb = oracle.preprocess(Fp, g, o_s, spec.in_scale)
    assert np.array_equal(xa, xb)
    # and the transposed-index mistake would not
    if h == wd:  # pragma: no cover
        pytest.skip("square frame")


def test_offset_change_is_local(net):
    spec, w = net
    R = S.receptive_radius(spec)
    h, wd = 64, 72
    F = S.render_frames(1, h, wd, "tiny", 12)[0]
    g = np.full((h, wd), 0.5)
    o = np.full((h, wd), 100.0)
    base = oracle.net_maps(F, spec, w, g, o)
    y, x = 20, 47
    o2 = o.copy()
    o2[y, x] -= 50.0
    m = oracle.net_maps(F, spec, w, g, o2)
    diff = np.abs(m - base).max(axis=0)
    yy, xx = np.nonzero(diff)
    assert diff[y, x] > 0
    # the stem reaches 1 pixel and each block 2 d: R = 1 + 2 sum(d) exactly
    assert np.abs(yy - y).max() == R and np.abs(xx - x).max() == R


def test_preprocess_batch_with_maps_applies_per_frame(net):
    spec, _ = net
    rng = np.random.default_rng(13)
    F = rng.integers(80, 300, size=(3, 9, 11)).astype(np.uint16)
    g = rng.uniform(0.4, 0.6, size=(9, 11))
    o = rng.uniform(95, 105, size=(9, 11))
    x = oracle.preprocess(F, g, o, spec.in_scale)
    for f in range(3):
        assert np.array_equal(x[f], oracle.preprocess(F[f], g, o, spec.in_scale))
    # a scalar beside a map broadcasts
    assert np.array_equal(oracle.preprocess(F[0], 0.5, o, 1.0), oracle.preprocess(F[0], np.full((9, 11), 0.5), o, 1.0))
