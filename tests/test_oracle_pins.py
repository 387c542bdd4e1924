"""Pins of the FP64 oracle against facts fixed by the mathematics, independent
library routines and brute force -- never against the oracle itself.

Each pin is chosen so that a plausible mistake in the oracle (a flipped tap, a
wrong dilation, a missing bias, a residual in the wrong place, an off-by-one in
the border handling, a tie broken the wrong way) fails at least one test.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
import smlm_synth as S

torch = pytest.importorskip("torch")
F = torch.nn.functional


def rng(seed=0):
    return np.random.default_rng(seed)


# ------------------------------------------------------------------ conv
@pytest.mark.parametrize("d", [1, 2, 3, 5])
def test_conv_delta_input_reproduces_weights(d):
    """A unit impulse at (i0, j0) of channel c gives y[o][i0 - d u][j0 - d v] = W[o][c][u+1][v+1]
    (cross-correlation orientation, tap spacing d), zero elsewhere, taps falling
    outside the frame simply missing."""
    r = rng(d)
    cin, cout, h, w = 3, 4, 13, 17
    W = r.standard_normal((cout, cin, 3, 3))
    for (i0, j0, c) in [(6, 8, 1), (0, 0, 0), (12, 16, 2), (1, 15, 0)]:
        x = np.zeros((cin, h, w))
        x[c, i0, j0] = 1.0
        y = oracle.conv3x3(x, W, None, d)
        expect = np.zeros((cout, h, w))
        for u in (-1, 0, 1):
            for v in (-1, 0, 1):
                i, j = i0 - d * u, j0 - d * v
                if 0 <= i < h and 0 <= j < w:
                    expect[:, i, j] = W[:, c, u + 1, v + 1]
        assert np.array_equal(y, expect)


def test_conv_linearity_and_bias():
    r = rng(1)
    cin, cout, h, w, d = 5, 6, 20, 23, 2
    W = r.standard_normal((cout, cin, 3, 3))
    b = r.standard_normal(cout)
    x1, x2 = r.standard_normal((2, cin, h, w))
    a1, a2 = 1.75, -0.5
    lhs = oracle.conv3x3(a1 * x1 + a2 * x2, W, None, d)
    rhs = a1 * oracle.conv3x3(x1, W, None, d) + a2 * oracle.conv3x3(x2, W, None, d)
    assert np.allclose(lhs, rhs, rtol=1e-12, atol=1e-12)
    yb = oracle.conv3x3(x1, W, b, d) - oracle.conv3x3(x1, W, None, d)
    assert np.allclose(yb, b[:, None, None] * np.ones((1, h, w)), atol=1e-12)


def test_conv_constant_field():
    """Constant input c: interior outputs are b + c * sum(W[o]); at the border only
    in-frame taps count."""
    r = rng(2)
    cin, cout, h, w, d = 2, 3, 16, 16, 4
    W = r.standard_normal((cout, cin, 3, 3))
    b = r.standard_normal(cout)
    c = 1.5
    y = oracle.conv3x3(np.full((cin, h, w), c), W, b, d)
    interior = b + c * W.sum(axis=(1, 2, 3))
    assert np.allclose(y[:, d:h - d, d:w - d], interior[:, None, None], rtol=1e-13)
    # corner (0, 0): only taps u, v in {0, +1} are inside
    corner = b + c * W[:, :, 1:, 1:].sum(axis=(1, 2, 3))
    assert np.allclose(y[:, 0, 0], corner, rtol=1e-13)


@pytest.mark.parametrize("d", [1, 2, 4, 8, 16])
def test_conv_matches_torch_float64(d):
    r = rng(10 + d)
    cin, cout, h, w = 4, 5, 37, 41
    x = r.standard_normal((cin, h, w))
    W = r.standard_normal((cout, cin, 3, 3))
    b = r.standard_normal(cout)
    ref = F.conv2d(torch.from_numpy(x)[None], torch.from_numpy(W), torch.from_numpy(b),
                   padding=d, dilation=d)[0].numpy()
    got = oracle.conv3x3(x, W, b, d)
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-12)


# ------------------------------------------------------------------- net
def torch_net(frame, spec, wts, gain=0.5, offset=100.0):
    """Independent float64 composition with torch.nn.functional (test-only)."""
    t = lambda k: torch.from_numpy(np.asarray(wts[k], np.float64))
    x = (torch.from_numpy(frame.astype(np.float64)) - offset) * gain * spec.in_scale
    a = F.relu(F.conv2d(x[None, None], t("stem.w"), t("stem.b"), padding=1))
    for k, d in enumerate(spec.dilations):
        tt = F.relu(F.conv2d(a, t(f"blk{k}.w1"), t(f"blk{k}.b1"), padding=d, dilation=d))
        a = F.relu(a + F.conv2d(tt, t(f"blk{k}.w2"), t(f"blk{k}.b2"), padding=d, dilation=d))
    m = torch.einsum("qc,nchw->nqhw", t("head.w"), a) + t("head.b")[None, :, None, None]
    return m[0].numpy()


@pytest.mark.parametrize("name", ["A", "B"])
def test_net_matches_torch_composition(name):
    spec = S.NETS[name]
    _, w = S.make_net(spec, seed=5, calibrated=False, bias_std=0.1)
    fr = S.render_frames(1, 48, 56, "tiny", 77)[0]
    got = oracle.net_maps(fr, spec, w)
    ref = torch_net(fr, spec, w)
    assert np.allclose(got, ref, rtol=1e-10, atol=1e-10)


def test_net_positive_homogeneity_exact():
    """With every bias zero, the network is positively homogeneous; doubling the
    gain doubles every map bit for bit (power-of-two scaling is exact)."""
    spec = S.NET_A
    _, w = S.make_net(spec, seed=3, calibrated=False)
    w["head.b"] = np.zeros(5, np.float32)
    fr = S.render_frames(1, 40, 40, "tiny", 5)[0]
    m1 = oracle.net_maps(fr, spec, w, gain=0.5)
    m2 = oracle.net_maps(fr, spec, w, gain=1.0)
    assert np.array_equal(m2, 2.0 * m1)
    assert np.abs(m1).max() > 0


def test_net_zero_blocks_reduce_to_stem_and_head():
    """Zero block weights and biases make every residual block the identity on
    non-negative inputs, so maps = head(ReLU(stem(x)))."""
    spec = S.NetSpec("z", 16, (1, 3))
    r = rng(4)
    w = {n: np.zeros(s, np.float32) for n, s in S.tensor_layout(spec)}
    w["stem.w"] = r.standard_normal((16, 1, 3, 3)).astype(np.float32)
    w["stem.b"] = r.standard_normal(16).astype(np.float32)
    w["head.w"] = r.standard_normal((5, 16)).astype(np.float32)
    w["head.b"] = r.standard_normal(5).astype(np.float32)
    fr = S.render_frames(1, 24, 30, "tiny", 6)[0]
    got = oracle.net_maps(fr, spec, w)
    x = (fr.astype(np.float64) - 100.0) * 0.5 * spec.in_scale
    a = F.relu(F.conv2d(torch.from_numpy(x)[None, None], torch.from_numpy(w["stem.w"].astype(np.float64)),
                        torch.from_numpy(w["stem.b"].astype(np.float64)), padding=1))[0].numpy()
    ref = np.einsum("qc,chw->qhw", w["head.w"].astype(np.float64), a) + w["head.b"].astype(np.float64)[:, None, None]
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("name", ["A", "B"])
def test_locality_receptive_radius(name):
    """Maps inside a window depend only on pixels within R = 1 + 2 sum(d) of it:
    a crop with an R margin reproduces the whole-frame maps bit for bit, and a
    crop with R - 1 does not (so the dilations really are used)."""
    spec = S.NETS[name]
    _, w = S.make_net(spec, seed=8, calibrated=False, bias_std=0.05)
    R = S.receptive_radius(spec)
    H = Wd = 2 * R + 40
    fr = S.render_frames(1, H, Wd, "tiny", 9)[0]
    full = oracle.net_maps(fr, spec, w)
    y0, x0, hh, ww = R + 3, R + 5, 20, 24
    win = oracle.net_maps_window(fr, spec, w, y0, x0, hh, ww)
    assert np.array_equal(win, full[:, y0:y0 + hh, x0:x0 + ww])
    short = oracle.net_maps_window(fr, spec, w, y0, x0, hh, ww, margin=R - 1)
    assert not np.allclose(short, full[:, y0:y0 + hh, x0:x0 + ww], rtol=1e-9, atol=1e-9)


def test_preprocess_closed_form():
    F16 = np.array([[0, 100, 101, 300, 65535]], np.uint16)
    x = oracle.preprocess(F16, gain=0.5, offset=100.0, in_scale=0.01)
    assert np.allclose(x, [[-0.5, 0.0, 0.005, 1.0, (65535 - 100) * 0.005]], rtol=1e-15, atol=1e-15)
    allv = np.arange(65536, dtype=np.uint16)[None]
    x = oracle.preprocess(allv, 0.5, 100.0, 0.01)
    assert np.allclose(np.diff(x), 0.005, rtol=1e-9)   # affine in the ADU


def test_param_counts_closed_form():
    assert S.param_count(S.NET_A) == 55973
    assert S.param_count(S.NET_B) == 208565
    assert S.net_flops_per_px(S.NET_A) == 111488
    assert S.net_flops_per_px(S.NET_B) == 416064
    assert S.receptive_radius(S.NET_A) == 15 and S.receptive_radius(S.NET_B) == 63


# -------------------------------------------------------------- detection
def brute_detect(L, tau):
    """Direct definition: a pixel is detected iff it exceeds tau and its key
    (value, -raster index) is the maximum key of its in-frame 3x3 neighbourhood."""
    h, w = L.shape
    out = np.zeros((h, w), bool)
    for i in range(h):
        for j in range(w):
            keys = [(L[a, b], -(a * w + b)) for a in range(max(0, i - 1), min(h, i + 2))
                    for b in range(max(0, j - 1), min(w, j + 2))]
            out[i, j] = L[i, j] > tau and max(keys) == (L[i, j], -(i * w + j))
    return out


def test_detect_exhaustive_3x3():
    """All 3^9 frames of size 3x3 over {0, 1, 2} with tau = 0.5."""
    vals = np.array(list(itertools.product((0.0, 1.0, 2.0), repeat=9)))
    for v in vals:
        L = v.reshape(3, 3)
        assert np.array_equal(oracle.detect(L, 0.5), brute_detect(L, 0.5)), L


def test_detect_random_plateaus_and_borders():
    r = rng(11)
    for k in range(60):
        h, w = r.integers(1, 9, size=2)
        L = r.integers(0, 4, size=(h, w)).astype(np.float64)   # many ties
        got = oracle.detect(L, 0.5)
        assert np.array_equal(got, brute_detect(L, 0.5))
        ii, jj = np.nonzero(got)                               # no two detections touch
        for a, b in zip(ii, jj):
            nb = got[max(0, a - 1):a + 2, max(0, b - 1):b + 2]
            assert nb.sum() == 1


def test_detect_constant_frame_single_winner():
    for h, w in [(1, 1), (1, 7), (5, 1), (6, 9)]:
        det = oracle.detect(np.full((h, w), 3.0), 0.0)
        assert det.sum() == 1 and det[0, 0]
        assert oracle.detect(np.full((h, w), -3.0), 0.0).sum() == 0


def test_detect_matches_maximum_filter_without_ties():
    ndimage = pytest.importorskip("scipy.ndimage")
    r = rng(12)
    L = r.standard_normal((64, 80))
    tau = 0.3
    mx = ndimage.maximum_filter(L, size=3, mode="constant", cval=-np.inf)
    ref = (L == mx) & (L > tau)
    assert np.array_equal(oracle.detect(L, tau), ref)


def test_threshold_is_probability_0_3():
    assert abs(1.0 / (1.0 + math.exp(-oracle.TAU)) - 0.3) < 1e-15
    assert abs(oracle.TAU - (-0.8472978603872037)) < 1e-15


@pytest.mark.parametrize("threshold", [0.3, 0.7])
def test_localize_threshold_is_a_probability(threshold):
    """The whole path keeps exactly the local maxima (found with no threshold)
    whose probability 1 / (1 + e^-logit) exceeds the threshold, at any threshold."""
    spec, w = S.make_net("A", 1)
    fr = S.render_frames(1, 64, 64, "tiny", 12)
    rec, maps = oracle.localize(fr, spec, w, threshold=threshold, return_maps=True)
    L = maps[0, 0]
    expect = oracle.detect(L, -np.inf) & (1.0 / (1.0 + np.exp(-L)) > threshold)
    assert len(rec) == expect.sum() > 0
    assert np.array_equal(np.stack([rec["row"], rec["col"]], 1), np.argwhere(expect))
    assert np.all(rec["prob"] > threshold)


def test_records_coordinates():
    spec = S.NET_A
    h, w = 4, 5
    maps = np.zeros((5, h, w))
    maps[:, 2, 3] = [2.0, 0.25, -0.125, 0.5, 1.5]
    det = np.zeros((h, w), bool)
    det[2, 3] = True
    rec = oracle.records(maps, det, spec, frame=7)
    assert rec.size == 1
    e = rec[0]
    assert (e["frame"], e["row"], e["col"]) == (7, 2, 3)
    assert e["x"] == 3 + 0.5 + 0.25 and e["y"] == 2 + 0.5 - 0.125
    assert e["z"] == 0.5 * spec.z_scale and e["photons"] == 1.5 * spec.ph_scale
    assert abs(e["prob"] - 1 / (1 + math.exp(-2.0))) < 1e-15


def test_localize_orders_by_frame_row_col():
    spec, w = S.make_net("A", 1)
    fr = S.render_frames(2, 64, 64, "tiny", 3)
    rec = oracle.localize(fr, spec, w)
    keys = list(zip(rec["frame"], rec["row"], rec["col"]))
    assert keys == sorted(keys) and len(set(keys)) == len(keys)


# --------------------------------------------------------------- rounding
def test_bf16_rounding_matches_torch():
    r = rng(13)
    v = np.concatenate([r.standard_normal(5000) * 10.0 ** r.integers(-6, 6, 5000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.005859375, 256.0, 257.0, 259.0, 65535.0]])
    v32 = v.astype(np.float32).astype(np.float64)
    ref = torch.from_numpy(v32).float().to(torch.bfloat16).double().numpy()
    assert np.array_equal(oracle.round_bf16(v32), ref)
    assert oracle.round_bf16(np.array([257.0]))[0] == 256.0     # tie to even
    assert oracle.round_bf16(np.array([259.0]))[0] == 260.0


def test_e4m3_rounding_codes_and_ties():
    codes = torch.arange(256, dtype=torch.uint8).view(torch.float8_e4m3fn).double().numpy()
    finite = codes[np.isfinite(codes)]
    assert np.array_equal(oracle.round_e4m3(finite), finite)          # every code is a fixed point
    pos = np.unique(finite[finite >= 0])
    assert pos.max() == 448.0 and pos[1] == 2.0 ** -9
    mids = 0.5 * (pos[1:] + pos[:-1])
    got = oracle.round_e4m3(mids)
    ref = torch.from_numpy(mids).float().to(torch.float8_e4m3fn).double().numpy()
    assert np.array_equal(got, ref)                                   # ties to even
    r = rng(14)
    v = r.standard_normal(20000) * 10.0 ** r.uniform(-3, 2.6, 20000)
    v = v[np.abs(v) < 464]
    ref = torch.from_numpy(v).float().to(torch.float8_e4m3fn).double().numpy()
    assert np.array_equal(oracle.round_e4m3(v.astype(np.float32).astype(np.float64)), ref)
    assert list(oracle.round_e4m3(np.array([500.0, -1e9, 448.0]))) == [448.0, -448.0, 448.0]


def test_bf16_mode_equals_exact_when_everything_is_representable():
    """Small-integer weights and inputs keep every stored activation an integer
    below 256, which bfloat16 represents exactly: BF16 emulation == exact."""
    spec = S.NetSpec("i", 16, (1, 2), in_scale=1.0)
    r = rng(15)
    w = {}
    for n, s in S.tensor_layout(spec):
        if n.endswith(("w", "w1", "w2")):
            w[n] = (r.integers(-1, 2, size=s) * (r.random(s) < 0.15)).astype(np.float32)
        else:
            w[n] = r.integers(-1, 2, size=s).astype(np.float32)
    fr = (100 + r.integers(0, 3, size=(20, 24))).astype(np.uint16)     # x in {0, 1, 2} with gain 1
    ex = oracle.net_maps(fr, spec, w, gain=1.0, offset=100.0, quant="exact")
    bf = oracle.net_maps(fr, spec, w, gain=1.0, offset=100.0, quant="bf16")
    assert np.abs(ex).max() < 256
    assert np.array_equal(ex, bf)


def test_bf16_mode_rounds_stored_activations():
    """One stem channel producing 257 (not a bfloat16 value) reaches the head as
    256 in BF16 mode (round to nearest even) and as 257 exactly."""
    spec = S.NetSpec("r", 16, (1,), in_scale=1.0)
    w = {n: np.zeros(s, np.float32) for n, s in S.tensor_layout(spec)}
    w["stem.w"][0, 0, 1, 1] = 1.0
    w["head.w"][0, 0] = 1.0
    fr = np.full((3, 3), 100 + 257, np.uint16)
    ex = oracle.net_maps(fr, spec, w, gain=1.0, offset=100.0)
    bf = oracle.net_maps(fr, spec, w, gain=1.0, offset=100.0, quant="bf16")
    assert ex[0, 1, 1] == 257.0 and bf[0, 1, 1] == 256.0


# ------------------------------------------------------------------- gate
def test_bce_closed_forms():
    L, dg = oracle.bce(np.array([0.0, 0.0]), np.array([1.0, 0.0]))
    assert abs(L - math.log(2.0)) < 1e-15
    assert np.allclose(dg, [-0.25, 0.25])
    g = np.array([40.0, -40.0, 3.0])
    y = np.array([1.0, 0.0, 1.0])
    L, dg = oracle.bce(g, y)
    expect = (math.log1p(math.exp(-40)) * 2 + math.log1p(math.exp(-3))) / 3
    assert abs(L - expect) < 1e-15
    assert np.allclose(dg, (1 / (1 + np.exp(-g)) - y) / 3, rtol=1e-14)


def _gate_problem(seed=0, n=3, size=8):
    r = rng(seed)
    theta = S.gate_flat(S.gate_init(seed)).astype(np.float64)
    theta[72:80] = r.standard_normal(8) * 0.1      # non-zero biases so every path is exercised
    theta[656:664] = r.standard_normal(8) * 0.1
    pooled = r.standard_normal((n, size, size))
    y = (r.random(n) < 0.5).astype(np.float64)
    return theta, pooled, y


def test_gate_gradient_central_differences():
    theta, pooled, y = _gate_problem()
    g = oracle.gate_forward(pooled, theta)
    _, dg = oracle.bce(g, y)
    grad = oracle.gate_backward(pooled, theta, dg)
    h = 1e-6
    for k in range(theta.size):
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        Lp, _ = oracle.bce(oracle.gate_forward(pooled, tp), y)
        Lm, _ = oracle.bce(oracle.gate_forward(pooled, tm), y)
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - grad[k]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (k, fd, grad[k])


def test_gate_forward_backward_match_torch_autograd():
    theta, pooled, y = _gate_problem(seed=1, n=4, size=16)
    t = torch.tensor(theta, requires_grad=True)
    w1, b1 = t[:72].view(8, 1, 3, 3), t[72:80]
    w2, b2 = t[80:656].view(8, 8, 3, 3), t[656:664]
    fw, fb = t[664:672], t[672]
    x = torch.from_numpy(pooled)[:, None]
    h1 = F.relu(F.conv2d(x, w1, b1, padding=1))
    h2 = F.relu(F.conv2d(h1, w2, b2, padding=1))
    g = h2.amax(dim=(2, 3)) @ fw + fb
    L = F.binary_cross_entropy_with_logits(g, torch.from_numpy(y))
    L.backward()
    go = oracle.gate_forward(pooled, theta)
    Lo, dg = oracle.bce(go, y)
    assert np.allclose(go, g.detach().numpy(), rtol=1e-12, atol=1e-12)
    assert abs(Lo - L.item()) < 1e-12
    assert np.allclose(oracle.gate_backward(pooled, theta, dg), t.grad.numpy(), rtol=1e-10, atol=1e-12)


def _identity_gate(fw0=2.0, fb=-1.0):
    """Gate whose channel 0 passes the pooled tile through two identity
    convolutions (h2[0] = ReLU(p)); every other channel is zero."""
    theta = np.zeros(673)
    theta[0 * 9 + 4] = 1.0                     # W1[0][0][1][1]
    theta[80 + (0 * 8 + 0) * 9 + 4] = 1.0      # W2[0][0][1][1]
    theta[664] = fw0
    theta[672] = fb
    return theta


def test_gate_global_pool_is_max_closed_form():
    r = rng(21)
    pooled = r.standard_normal((3, 8, 8))
    theta = _identity_gate()
    g = oracle.gate_forward(pooled, theta)
    expect = 2.0 * np.maximum(pooled, 0).reshape(3, -1).max(axis=1) - 1.0
    assert np.allclose(g, expect, rtol=0, atol=1e-15)


def test_gate_max_gradient_goes_to_first_maximum():
    p = np.zeros((1, 8, 8))
    p[0, 2, 3] = p[0, 5, 6] = 1.5               # a tie; (2, 3) comes first in raster order
    p[0, 2, 4] = 0.25                           # neighbours that tell the two apart
    p[0, 6, 6] = 0.75
    theta = _identity_gate()
    grad = oracle.gate_backward(p, theta, np.array([1.0]))
    first, second = p.copy(), p.copy()
    second[0, 2, 3] -= 1e-3                     # only (5, 6) attains the max
    first[0, 5, 6] -= 1e-3                      # only (2, 3) attains the max
    g_first = oracle.gate_backward(first, theta, np.array([1.0]))
    g_second = oracle.gate_backward(second, theta, np.array([1.0]))
    w2 = slice(80, 89)                          # dW2[0][0][:][:] = fw0 * h1 around the argmax
    assert np.allclose(grad[w2], g_first[w2], atol=1e-12)
    assert not np.allclose(grad[w2], g_second[w2], atol=1e-3)
    assert grad[80 + 5] == 2.0 * 0.25 and g_second[80 + 7] == 2.0 * 0.75


def test_gate_pool_mean_of_blocks():
    x = np.arange(64, dtype=np.float64).reshape(8, 8)
    p = oracle.gate_pool(x, 4)
    assert p.shape == (2, 2)
    assert p[0, 0] == np.mean(x[:4, :4]) and p[1, 1] == np.mean(x[4:, 4:])


def test_adam_matches_torch():
    r = rng(16)
    theta = r.standard_normal(673)
    m = np.zeros(673)
    v = np.zeros(673)
    tt = torch.tensor(theta.copy(), requires_grad=True)
    opt = torch.optim.Adam([tt], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    for step in range(1, 6):
        g = r.standard_normal(673)
        oracle.adam_step(theta, m, v, g, step)
        opt.zero_grad()
        tt.grad = torch.from_numpy(g.copy())
        opt.step()
    assert np.allclose(theta, tt.detach().numpy(), rtol=1e-12, atol=1e-14)


# ------------------------------------------------------------ FP8 storage
def test_fp8_group_exponent_is_smallest_fitting_power_of_two():
    r = rng(31)
    vals = np.concatenate([r.lognormal(0, 3, 2000), [448.0, 448.0000001, 224.0, 1.0, 1.75, 1.7500001, 3.5e-30]])
    for a in vals:
        k = oracle.fp8_group_exp(a)
        assert a <= 448.0 * 2.0 ** k and not a <= 448.0 * 2.0 ** (k - 1), (a, k)
    assert oracle.fp8_group_exp(0.0) == -126


def test_fp8_group_storage_brute_force():
    r = rng(32)
    C, n = 48, 300
    a = np.abs(r.standard_normal((C, n))) * np.exp(r.uniform(-6, 6, n))[None, :]
    got = oracle.store_fp8_groups(a)
    b = a
    for p in range(n):
        for c0, c1 in ((0, 32), (32, 48)):
            amax = np.max(np.abs(b[c0:c1, p]))
            k = next(k for k in range(-140, 140) if amax <= 448.0 * 2.0 ** k)    # smallest fitting scale
            k = max(k, -126)
            expect = oracle.round_e4m3(b[c0:c1, p] / 2.0 ** k) * 2.0 ** k
            assert np.array_equal(got[c0:c1, p], expect)
            assert np.max(np.abs(got[c0:c1, p])) <= 448.0 * 2.0 ** k


def test_fp8_group_storage_scale_invariant_and_exact_on_codes():
    r = rng(33)
    a = np.abs(r.standard_normal((40, 64)))
    q = oracle.store_fp8_groups(a)
    assert np.array_equal(oracle.store_fp8_groups(q), q)              # stored values are fixed points
    assert np.array_equal(oracle.store_fp8_groups(a * 2.0 ** 9), q * 2.0 ** 9)   # power-of-two scaling commutes
    assert np.max(np.abs(q - a) / np.maximum(np.abs(a), 1e-3)) < 0.07  # e4m3: 3 mantissa bits
