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
