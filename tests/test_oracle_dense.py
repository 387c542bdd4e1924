"""Pins of the oracle's dense-connection dilated network (paper Sec. 3.2 /
3.2.1: each layer of a block uses the outputs of all earlier layers; Sec.
4.1.2: dilations 2, 4, 8, 16):

* the whole network against an independent torch float64 composition
  (torch.cat for the concatenations, conv2d with dilation, 1x1 transitions
  and head), random biases everywhere;
* locality: a crop with the receptive radius 1 + L * sum(d) as margin
  reproduces the frame's maps exactly, one pixel less does not;
* parameter and FLOP counts against closed forms written out here;
* blocks whose layers are zero and whose transitions copy the block input
  reduce the network to stem + head, bit for bit equal to the residual
  oracle with no blocks.

The two-stage U-Net stage after the blocks (Sec. 3.2: a two-stage U-Net
refines the extracted features; its sizes are a reading):

* against the same torch composition extended with max_pool2d (ceil mode),
  nearest interpolation and torch.cat, on frames of odd and even sides;
* a U-Net whose up convolution at level 0 copies the skip input and whose
  other convolutions are zero reduces the net to the one without it, bit for
  bit;
* its reach: changing one input pixel changes outputs up to the receptive
  radius 1 + L * sum(d) + 12 away and none farther; crops aligned to 4 pixels
  with that margin are exact, a crop shifted by one pixel is not.
"""
import numpy as np
import pytest

import oracle
import smlm_synth as S

torch = pytest.importorskip("torch")
F = torch.nn.functional


def torch_dense(frame, spec, w, gain=0.5, offset=100.0):
    t = lambda k: torch.from_numpy(np.asarray(w[k], np.float64))
    x = (torch.from_numpy(frame.astype(np.float64)) - offset) * gain * spec.in_scale
    a = F.relu(F.conv2d(x[None, None], t("stem.w"), t("stem.b"), padding=1))
    for k, d in enumerate(spec.dilations):
        cat = a
        for i in range(spec.layers):
            y = F.relu(F.conv2d(cat, t(f"blk{k}.l{i}.w"), t(f"blk{k}.l{i}.b"), padding=d, dilation=d))
            cat = torch.cat([cat, y], dim=1)
        a = F.relu(F.conv2d(cat, t(f"blk{k}.t.w")[:, :, None, None], t(f"blk{k}.t.b")))
    if getattr(spec, "unet", 0):
        h, w_ = a.shape[2], a.shape[3]
        h1, w1 = -(-h // 2), -(-w_ // 2)

        def up(v, hh, ww):
            return F.interpolate(v, scale_factor=2, mode="nearest")[:, :, :hh, :ww]
        conv = lambda v, k: F.relu(F.conv2d(v, t(f"unet.{k}.w"), t(f"unet.{k}.b"), padding=1))
        d1 = conv(F.max_pool2d(a, 2, ceil_mode=True), "d1")
        d2 = conv(F.max_pool2d(d1, 2, ceil_mode=True), "d2")
        u1 = conv(torch.cat([d1, up(d2, h1, w1)], dim=1), "u1")
        a = conv(torch.cat([a, up(u1, h, w_)], dim=1), "u0")
    m = F.conv2d(a, t("head.w")[:, :, None, None], t("head.b"))
    return m[0].numpy()


@pytest.mark.parametrize("spec", [S.NET_D, S.DenseSpec("d2", 16, (1, 3), layers=3, growth=8)])
def test_dense_net_matches_torch_composition(spec):
    w = S.he_normal_weights(spec, 12, bias_std=0.1)
    fr = S.render_frames(1, 41, 57, "tiny", 81)[0]
    got = oracle.net_maps(fr, spec, w)
    ref = torch_dense(fr, spec, w)
    scale = np.sqrt(np.mean(ref ** 2, axis=(1, 2)))[:, None, None]
    assert np.max(np.abs(got - ref) / (np.abs(ref) + scale)) <= 1e-12


def test_dense_net_locality():
    spec = S.DenseSpec("d3", 16, (2, 3), layers=2, growth=8)
    w = S.he_normal_weights(spec, 13, bias_std=0.05)
    R = S.receptive_radius(spec)
    assert R == 1 + 2 * (2 + 3)
    fr = S.render_frames(1, 60, 64, "tiny", 82)[0]
    full = oracle.net_maps(fr, spec, w)
    y0, x0, hh, ww = 24, 26, 6, 7
    win = oracle.net_maps_window(fr, spec, w, y0, x0, hh, ww)
    assert np.array_equal(win, full[:, y0:y0 + hh, x0:x0 + ww])
    short = oracle.net_maps_window(fr, spec, w, y0, x0, hh, ww, margin=R - 1)
    assert not np.array_equal(short, full[:, y0:y0 + hh, x0:x0 + ww])


def test_dense_counts_closed_form():
    C, G, L, B, nh = 32, 16, 4, 4, 5
    params = (9 * C + C) + B * (sum(9 * (C + i * G) * G + G for i in range(L)) + (C + L * G) * C + C) + nh * C + nh
    assert params == S.param_count(S.NET_D) == 142181
    flop = 2 * (9 * C + B * (sum(9 * (C + i * G) * G for i in range(L)) + (C + L * G) * C) + nh * C)
    assert flop == S.net_flops_per_px(S.NET_D) == 283520
    assert S.receptive_radius(S.NET_D) == 1 + 4 * (2 + 4 + 8 + 16)


def test_identity_blocks_reduce_to_stem_and_head():
    spec = S.DenseSpec("d4", 16, (2, 4), layers=2, growth=8)
    w = S.he_normal_weights(spec, 14, bias_std=0.1)
    for k in range(len(spec.dilations)):
        for i in range(spec.layers):
            w[f"blk{k}.l{i}.w"][:] = 0
            w[f"blk{k}.l{i}.b"][:] = 0
        tw = np.zeros_like(w[f"blk{k}.t.w"])
        tw[:, :spec.C] = np.eye(spec.C, dtype=np.float32)
        w[f"blk{k}.t.w"] = tw
        w[f"blk{k}.t.b"][:] = 0
    fr = S.render_frames(1, 33, 29, "tiny", 83)[0]
    base = S.NetSpec("r0", spec.C, ())
    wb = {"stem.w": w["stem.w"], "stem.b": w["stem.b"], "head.w": w["head.w"], "head.b": w["head.b"]}
    assert np.array_equal(oracle.net_maps(fr, spec, w), oracle.net_maps(fr, base, wb))


UNET_SMALL = S.DenseSpec("u2", 16, (1, 2), layers=2, growth=16, unet=2)


@pytest.mark.parametrize("spec,h,w", [(S.NET_DU, 41, 57), (UNET_SMALL, 38, 29), (UNET_SMALL, 5, 3), (UNET_SMALL, 1, 1)])
def test_unet_matches_torch_composition(spec, h, w):
    wts = S.he_normal_weights(spec, 15, bias_std=0.1)
    fr = S.render_frames(1, h, w, "tiny", 84)[0]
    got = oracle.net_maps(fr, spec, wts)
    ref = torch_dense(fr, spec, wts)
    scale = np.sqrt(np.mean(ref ** 2, axis=(1, 2)))[:, None, None] + 1e-300
    assert np.max(np.abs(got - ref) / (np.abs(ref) + scale)) <= 1e-12


def test_unet_with_a_skip_copy_reduces_to_the_net_without_it():
    spec = UNET_SMALL
    plain = S.DenseSpec("u0", 16, (1, 2), layers=2, growth=16)
    w = S.he_normal_weights(spec, 16, bias_std=0.1)
    C = spec.C
    for k in ("d1", "d2", "u1", "u0"):
        w[f"unet.{k}.w"] = np.zeros_like(w[f"unet.{k}.w"])
        w[f"unet.{k}.b"] = np.zeros_like(w[f"unet.{k}.b"])
    w["unet.u0.w"][np.arange(C), np.arange(C), 1, 1] = 1.0        # u0 = ReLU(a0) = a0
    wp = {k: v for k, v in w.items() if not k.startswith("unet.")}
    fr = S.render_frames(1, 37, 44, "tiny", 85)[0]
    assert np.array_equal(oracle.net_maps(fr, spec, w), oracle.net_maps(fr, plain, wp))


def test_unet_reach_and_crop_alignment():
    spec = UNET_SMALL
    R = S.receptive_radius(spec)
    assert oracle.unet_reach(spec) == S.UNET_REACH == 12 and R == 1 + 2 * (1 + 2) + 12
    w = S.he_normal_weights(spec, 17, bias_std=0.2)
    fr = S.render_frames(1, 72, 80, "tiny", 86)[0].astype(np.int64)
    base = oracle.net_maps(fr.astype(np.uint16), spec, w)
    seen = 0
    for (y, x) in [(36, 40), (37, 41), (38, 42), (39, 43)]:     # every phase modulo 4
        g = fr.copy()
        g[y, x] += 500
        diff = np.any(oracle.net_maps(g.astype(np.uint16), spec, w) != base, axis=0)
        yy, xx = np.nonzero(diff)
        dist = np.maximum(np.abs(yy - y), np.abs(xx - x))
        assert dist.max() <= R                       # nothing farther than the radius changes
        seen = max(seen, int(dist.max()))
    assert seen == R                                 # and the radius is reached
    f16 = fr.astype(np.uint16)
    y0, x0, hh, ww = 30, 33, 9, 11
    assert np.array_equal(oracle.net_maps_window(f16, spec, w, y0, x0, hh, ww), base[:, y0:y0 + hh, x0:x0 + ww])
    # the same crop shifted by one pixel moves the pooling windows
    cy0, cx0 = (y0 - R) // 4 * 4 + 1, (x0 - R) // 4 * 4 + 1
    crop = oracle.net_maps(f16[cy0:y0 + hh + R, cx0:x0 + ww + R], spec, w)
    assert not np.array_equal(crop[:, y0 - cy0:y0 - cy0 + hh, x0 - cx0:x0 - cx0 + ww], base[:, y0:y0 + hh, x0:x0 + ww])


def test_unet_counts_closed_form():
    C, G, L, B, nh = 32, 16, 4, 4, 5
    unet = 9 * C * C + C + 9 * C * C + C + 9 * 2 * C * C + C + 9 * 2 * C * C + C
    assert S.param_count(S.NET_DU) == S.param_count(S.NET_D) + unet == 197605
    assert S.net_flops_per_px(S.NET_DU) == S.net_flops_per_px(S.NET_D) + 2 * 9 * C * C * (1 / 4 + 1 / 16 + 2 / 4 + 2)
