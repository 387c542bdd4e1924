"""Pins of the oracle's FP8 emulation, against facts fixed outside it.

* Weight quantisation (one scale per output channel, max|W[o]| / 448): a
  channel whose weights are its maximum times e4m3 values over 448 comes back
  exactly (up to the FP32 rounding of its scale), whatever the other channels
  hold; scaling one channel by a power of two scales its quantised weights by
  the same power and leaves every other channel bit for bit; the result equals
  torch's own float8_e4m3fn cast of the scaled FP32 weights.
* Where the activation scales sit: the FP8 network equals an independent
  torch float64 composition that stores the stem output, every block's
  intermediate and every block output but the last as e4m3 values with one
  power-of-two scale per 32-channel group of each pixel.  Its rounding to
  e4m3 is a nearest-value search over torch's table of the 256 codes (ties to
  the even code), not the oracle's routine.
"""
import numpy as np
import pytest

import oracle
import smlm_synth as S

torch = pytest.importorskip("torch")
F = torch.nn.functional


def rng(seed=0):
    return np.random.default_rng(seed)


def e4m3_table():
    """The finite e4m3fn values and their code integers, ascending by value."""
    codes = torch.arange(256, dtype=torch.uint8)
    vals = codes.view(torch.float8_e4m3fn).double().numpy()
    ok = np.isfinite(vals) & ~((vals == 0) & np.signbit(vals))      # one zero
    v, c = vals[ok], codes.numpy()[ok].astype(np.int64)
    order = np.argsort(v)
    return v[order], c[order]


_TABLE = e4m3_table()


def round_e4m3_search(x):
    """Nearest finite e4m3 value (ties to the even code integer), saturating
    at +-448: a search over the value table."""
    vals, codes = _TABLE
    x = np.clip(np.asarray(x, np.float64), vals[0], vals[-1])
    hi = np.clip(np.searchsorted(vals, x, side="left"), 1, len(vals) - 1)
    lo = hi - 1
    dlo, dhi = x - vals[lo], vals[hi] - x
    pick_hi = (dhi < dlo) | ((dhi == dlo) & (codes[hi] % 2 == 0))
    return np.where(pick_hi, vals[hi], vals[lo])


def quant_weights_torch(W):
    """Per-output-channel e4m3 quantisation with torch: codes of the FP32
    product W * fl32(448 / max|W[o]|), times the FP32 scale max|W[o]| / 448."""
    W = np.asarray(W, np.float64)
    out = np.zeros_like(W)
    for o in range(W.shape[0]):
        mx = np.max(np.abs(W[o]))
        if mx == 0:
            continue
        inv = torch.tensor(448.0 / mx, dtype=torch.float64).float()
        ws = torch.tensor(mx / 448.0, dtype=torch.float64).float().double()
        sc = torch.from_numpy(W[o]).float() * inv
        out[o] = (sc.to(torch.float8_e4m3fn).double() * ws).numpy()
    return out


# ---------------------------------------------------------- weight scales
def test_fp8_weight_quant_closed_form():
    """W[o] = m_o * c / 448 with c e4m3 values and |c| = 448 present: the
    dequantised weights equal W to the FP32 rounding of the scale, with
    channel maxima spread over 2^-14 .. 2^5 (a tensor-wide scale would crush
    the small channels onto a few codes)."""
    r = rng(41)
    vals = _TABLE[0]
    cout, per = 16, 9 * 12
    m = (2.0 ** r.uniform(-14, 5, cout)).astype(np.float32).astype(np.float64)
    c = r.choice(vals, (cout, per))
    c[:, 0] = np.where(r.random(cout) < 0.5, 448.0, -448.0)
    W = (m[:, None] * c / 448.0).astype(np.float32).astype(np.float64).reshape(cout, 12, 3, 3)
    q = oracle.quant_weights_fp8(W)
    assert np.all(np.abs(q - W) <= 2.0 ** -22 * np.abs(W))


def test_fp8_weight_quant_per_channel_properties():
    r = rng(42)
    W = (r.standard_normal((48, 48, 3, 3)) * np.sqrt(2 / 432)).astype(np.float32).astype(np.float64)
    W[5] *= 1e-3                                    # channels of very different size
    W[9] *= 40.0
    W = W.astype(np.float32).astype(np.float64)
    q = oracle.quant_weights_fp8(W)
    # equal to torch's own cast of the same FP32 arithmetic
    assert np.array_equal(q, quant_weights_torch(W))
    for o in range(48):
        mx = np.max(np.abs(W[o]))
        # the channel maximum survives; e4m3 keeps 3 mantissa bits on normal codes
        assert abs(np.max(np.abs(q[o])) - mx) <= 2.0 ** -22 * mx
        normal = np.abs(W[o]) * 448.0 / mx >= 2.0 ** -6
        err = np.abs(q[o] - W[o])[normal] / np.abs(W[o])[normal]
        assert err.max() <= 2.0 ** -4 * (1 + 1e-6)
    # scaling one channel by a power of two touches only that channel
    W2 = W.copy()
    W2[3] *= 2.0 ** 6
    W2[7] *= 2.0 ** -7
    q2 = oracle.quant_weights_fp8(W2)
    assert np.array_equal(q2[3], q[3] * 2.0 ** 6) and np.array_equal(q2[7], q[7] * 2.0 ** -7)
    rest = [o for o in range(48) if o not in (3, 7)]
    assert np.array_equal(q2[rest], q[rest])


# ------------------------------------------------- activation scale points
def store_groups_torch(a):
    """FP8 storage of [C][h][w]: per pixel and 32-channel group, the smallest
    power of two 2^k >= amax / 448 (k >= -126), values e4m3(v / 2^k) 2^k."""
    a = np.asarray(a, np.float64)
    out = a.copy()
    for c0 in range(0, a.shape[0], 32):
        g = a[c0:c0 + 32]
        amax = np.max(np.abs(g), axis=0)
        with np.errstate(divide="ignore"):
            k = np.ceil(np.log2(amax / 448.0))
        k = np.where(amax > 0, k, -126.0)
        # make k exact at powers of two whatever log2's last bit did
        k = np.where(amax > 448.0 * 2.0 ** k, k + 1, k)
        k = np.where(amax <= 448.0 * 2.0 ** (k - 1), k - 1, k)
        k = np.maximum(k, -126.0)
        s = 2.0 ** k
        out[c0:c0 + 32] = round_e4m3_search(g / s) * s
    return out


def torch_net_fp8(frame, spec, wts, gain=0.5, offset=100.0):
    t = lambda k: torch.from_numpy(np.asarray(wts[k], np.float64))
    tq = lambda k: torch.from_numpy(quant_weights_torch(np.asarray(wts[k], np.float64)))
    st = lambda x: torch.from_numpy(store_groups_torch(x[0].numpy()))[None]
    x = (torch.from_numpy(frame.astype(np.float64)) - offset) * gain * spec.in_scale
    a = F.relu(F.conv2d(x[None, None], t("stem.w"), t("stem.b"), padding=1))
    a = st(a)
    nb = len(spec.dilations)
    for k, d in enumerate(spec.dilations):
        tt = st(F.relu(F.conv2d(a, tq(f"blk{k}.w1"), t(f"blk{k}.b1"), padding=d, dilation=d)))
        a = F.relu(a + F.conv2d(tt, tq(f"blk{k}.w2"), t(f"blk{k}.b2"), padding=d, dilation=d))
        if k + 1 < nb:
            a = st(a)
    m = torch.einsum("qc,nchw->nqhw", t("head.w"), a) + t("head.b")[None, :, None, None]
    return m[0].numpy()


@pytest.mark.parametrize("C,dil", [(48, (1, 2, 4)), (40, (2, 1))])
def test_fp8_emulation_matches_torch_composition(C, dil):
    """C = 48 has a full and a 16-channel group per pixel; C = 40 a full and
    an 8-channel one.  Random biases keep every stored tensor non-trivial."""
    spec = S.NetSpec("q", C, dil)
    w = S.he_normal_weights(spec, 8, bias_std=0.1)
    fr = S.render_frames(1, 30, 38, "tiny", 78)[0]
    got = oracle.net_maps(fr, spec, w, quant="fp8")
    ref = torch_net_fp8(fr, spec, w)
    ex = oracle.net_maps(fr, spec, w)
    scale = np.sqrt(np.mean(ref ** 2, axis=(1, 2)))[:, None, None]
    assert np.max(np.abs(got - ref) / (np.abs(ref) + scale)) <= 1e-9
    assert np.max(np.abs(ex - ref) / (np.abs(ref) + scale)) > 1e-4      # the rounding is really there
