"""Pins of the oracle's split-BF16 emulation (quant "bf16x3"): activations
stored in FP32, each block-convolution product formed from BF16 halves as
wh xh + wh xl + wl xh (v = hi + lo, hi = bf16(v), lo = bf16(v - hi)).

* the split against torch's own bfloat16 casts, its closed-form error bound
  (|v - hi - lo| <= 2^-17 |v|) and exactness for values of <= 16 bits;
* the whole emulated network against an independent torch float64
  composition (torch casts for the split, torch conv2d for the sums);
* on a network whose weights and activations are all BF16 values (lo = 0)
  the emulation equals the exact oracle;
* its distance to the exact oracle stays within the analytic size of the
  dropped terms (and the rounding really is there).
"""
import numpy as np
import pytest

import oracle
import smlm_synth as S
from tests.exact_nets import max_intermediate

torch = pytest.importorskip("torch")
F = torch.nn.functional


def split_torch(v):
    f = torch.as_tensor(np.asarray(v, np.float64)).float()
    hi = f.bfloat16().float()
    lo = (f - hi).bfloat16().float()
    return hi.double(), lo.double()


def test_split_matches_torch_casts_and_error_bound():
    r = np.random.default_rng(4)
    v = np.concatenate([r.standard_normal(20000) * 10.0 ** r.integers(-6, 6, 20000),
                        [0.0, 1.0, -1.0, 3.0, 1.0 + 2.0 ** -8, 1.0 + 2.0 ** -15, 65535.0]])
    v = v.astype(np.float32).astype(np.float64)
    hi, lo = oracle.split_bf16(v)
    th, tl = split_torch(v)
    assert np.array_equal(hi, th.numpy()) and np.array_equal(lo, tl.numpy())
    assert np.all(np.abs(v - hi - lo) <= 2.0 ** -17 * np.abs(v))
    # 16 significant bits or fewer: the pair is exact
    ints = r.integers(-(2 ** 16), 2 ** 16, 5000).astype(np.float64)
    h2, l2 = oracle.split_bf16(ints)
    assert np.array_equal(h2 + l2, ints)


def torch_net_bf16x3(frame, spec, wts, gain=0.5, offset=100.0):
    t = lambda k: torch.from_numpy(np.asarray(wts[k], np.float64))
    f32 = lambda x: x.float().double()

    def conv3(x, W, b, d):
        xh, xl = split_torch(x.numpy())
        wh, wl = split_torch(W.numpy())
        y = F.conv2d(xh, wh, b, padding=d, dilation=d)
        y = y + F.conv2d(xl, wh, None, padding=d, dilation=d)
        return y + F.conv2d(xh, wl, None, padding=d, dilation=d)

    x = (torch.from_numpy(frame.astype(np.float64)) - offset) * gain * spec.in_scale
    a = f32(F.relu(F.conv2d(x[None, None], t("stem.w"), t("stem.b"), padding=1)))
    for k, d in enumerate(spec.dilations):
        tt = f32(F.relu(conv3(a, t(f"blk{k}.w1"), t(f"blk{k}.b1"), d)))
        a = f32(F.relu(a + conv3(tt, t(f"blk{k}.w2"), t(f"blk{k}.b2"), d)))
    m = torch.einsum("qc,nchw->nqhw", t("head.w"), a) + t("head.b")[None, :, None, None]
    return m[0].numpy()


@pytest.mark.parametrize("C,dil", [(32, (1, 2, 4)), (16, (3, 1))])
def test_bf16x3_emulation_matches_torch_composition(C, dil):
    spec = S.NetSpec("s", C, dil)
    w = S.he_normal_weights(spec, 11, bias_std=0.1)
    fr = S.render_frames(1, 30, 41, "tiny", 79)[0]
    got = oracle.net_maps(fr, spec, w, quant="bf16x3")
    ref = torch_net_bf16x3(fr, spec, w)
    ex = oracle.net_maps(fr, spec, w)
    scale = np.sqrt(np.mean(ref ** 2, axis=(1, 2)))[:, None, None]
    e = np.abs(got - ref) / (np.abs(ref) + scale)
    # equal up to FP64 summation order: a sum that lands on the other side of
    # an FP32 (or BF16 split) rounding boundary in one of the two changes that
    # one stored value by an ulp, so a few outputs may differ at that size
    assert np.mean(e > 1e-12) < 0.01 and e.max() < 1e-6
    d = np.max(np.abs(ex - ref) / (np.abs(ref) + scale))
    assert 1e-8 < d < 1e-3                  # the split's rounding is there, and small


def test_bf16x3_equals_exact_on_bf16_valued_nets():
    """Weights and inputs of few bits keep every stored value a BF16 value
    (lo = 0 everywhere): the three-term product is then the exact product."""
    spec = S.NetSpec("i", 16, (1, 2), in_scale=1.0)
    r = np.random.default_rng(2)
    w = {}
    for n, s in S.tensor_layout(spec):
        p = 0.04 if n.endswith(("w1", "w2")) else 0.3
        w[n] = (r.integers(-1, 2, size=s) * (r.random(s) < p)).astype(np.float32)
    fr = (100 + r.integers(0, 3, size=(20, 24))).astype(np.uint16)
    ex = oracle.net_maps(fr, spec, w, gain=1.0, offset=100.0)
    # every value a block convolution reads is an integer below 256: 8 bits
    assert max_intermediate(fr, spec, w, include_head=False) < 256
    assert np.array_equal(oracle.net_maps(fr, spec, w, gain=1.0, offset=100.0, quant="bf16x3"), ex)
