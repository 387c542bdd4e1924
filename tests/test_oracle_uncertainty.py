"""Pins of the oracle's 10-output head (detection, offsets, photons, then the
raw uncertainties of x, y, z and photons and the background) and of the
softplus that turns raw uncertainties into positive values:

* softplus at special values and its identity softplus(u) - softplus(-u) = u;
* closed form of the head: with zero block weights and a stem that passes the
  input through channel 0, plane q is b_q + W[q][0] ReLU(x) exactly, so a
  transposed head matrix or a shifted bias fails;
* the five planes of the 5-output head are unchanged by the extra rows;
* units of the records' uncertainties at raw value 0 (softplus(0) = ln 2).
"""
import math

import numpy as np
import pytest

import oracle
import smlm_synth as S


def test_softplus_special_values():
    assert oracle.softplus(0.0) == pytest.approx(math.log(2.0), rel=1e-15)
    u = np.linspace(-30, 30, 601)
    assert np.allclose(oracle.softplus(u) - oracle.softplus(-u), u, rtol=0, atol=1e-13)
    assert oracle.softplus(40.0) == pytest.approx(40.0, rel=1e-16)
    # far below zero log(1 + e^u) = e^u (1 - e^u / 2 + ...): no underflow to 0
    assert oracle.softplus(-40.0) == pytest.approx(math.exp(-40.0), rel=1e-15)
    assert oracle.softplus(-800.0) == 0.0 and oracle.softplus(800.0) == 800.0
    assert np.all(np.diff(oracle.softplus(u)) > 0)


def _pass_through_net(spec, seed):
    rng = np.random.default_rng(seed)
    w = {k: np.zeros(s, np.float32) for k, s in S.tensor_layout(spec)}
    w["stem.w"][0, 0, 1, 1] = 1.0
    w["head.w"] = rng.standard_normal(w["head.w"].shape).astype(np.float32)
    w["head.b"] = rng.standard_normal(w["head.b"].shape).astype(np.float32)
    return w


@pytest.mark.parametrize("name", ["AU", "BU"])
def test_head_closed_form(name):
    spec = S.NETS[name]
    assert spec.head_outputs == 10
    w = _pass_through_net(spec, 3)
    F = S.render_frames(1, 33, 47, "tiny", 8)[0]
    m = oracle.net_maps(F, spec, w)
    x = np.maximum(oracle.preprocess(F, 0.5, 100.0, spec.in_scale), 0.0)
    Wh = w["head.w"].astype(np.float64)
    bh = w["head.b"].astype(np.float64)
    expect = bh[:, None, None] + Wh[:, 0][:, None, None] * x[None]
    assert m.shape == (10, 33, 47)
    assert np.allclose(m, expect, rtol=1e-14, atol=1e-14)


def test_extra_rows_leave_the_first_five_planes_alone():
    s5, w5 = S.make_net("A", 1)
    s10, w10 = S.make_net("AU", 1)
    F = S.render_frames(1, 40, 52, "tiny", 9)[0]
    m5 = oracle.net_maps(F, s5, w5)
    m10 = oracle.net_maps(F, s10, w10)
    assert np.array_equal(m10[:5], m5)
    assert np.all(np.isfinite(m10[5:]))


def test_uncertainty_units_at_zero_raw_value():
    spec = S.NETS["BU"]
    maps = np.zeros((10, 4, 5))
    det = np.zeros((4, 5), bool)
    det[1, 2] = det[3, 0] = True
    u = oracle.uncertainties(maps, det, spec)
    ln2 = math.log(2.0)
    s0 = ln2 + 0.01                      # a sigma at raw 0: softplus(0) plus the 0.01-unit floor
    assert len(u) == 2
    assert np.allclose(u["sigma_x"], s0) and np.allclose(u["sigma_y"], s0)
    assert np.allclose(u["sigma_z"], s0 * spec.z_scale)
    assert np.allclose(u["sigma_photons"], s0 * spec.ph_scale)
    assert np.allclose(u["background"], ln2 / spec.in_scale)


def test_localize_returns_matching_uncertainties():
    spec, w = S.make_net("AU", 1)
    frames = S.render_frames(2, 64, 72, "tiny", 10)
    rec, unc, maps = oracle.localize(frames, spec, w, with_uncertainty=True, return_maps=True)
    assert len(rec) == len(unc) > 0
    for r, q in zip(rec[:20], unc[:20]):
        raw = maps[r["frame"], 5:, r["row"], r["col"]]
        assert q["sigma_x"] == oracle.softplus(raw[0]) + 0.01
        assert q["background"] == oracle.softplus(raw[4]) / spec.in_scale
    # the 5-output net's records are those of the 10-output net
    s5, w5 = S.make_net("A", 1)
    assert np.array_equal(oracle.localize(frames, s5, w5), rec)


def test_sigma_filter_invariants():
    """The uncertainty filter only removes detections, the removed set grows as
    the limit falls (nested), nothing survives a limit below every sigma, a
    limit above every sigma changes nothing, and a removed maximum does not
    promote a neighbour (the survivors are a subset of the local maxima)."""
    spec, w = S.make_net("AU", 1)
    frames = S.render_frames(2, 96, 120, "tiny", 11)
    base, unc, maps = oracle.localize(frames, spec, w, with_uncertainty=True, return_maps=True)
    assert len(base) > 10
    sig = np.maximum(unc["sigma_x"], unc["sigma_y"])
    keys = lambda r: set(zip(r["frame"].tolist(), r["row"].tolist(), r["col"].tolist()))  # noqa: E731
    kb = keys(base)
    prev = kb
    for lim in sorted(set(np.quantile(sig, [0.9, 0.6, 0.3]).tolist()), reverse=True):
        r = oracle.localize(frames, spec, w, max_sigma_px=lim)
        k = keys(r)
        assert k <= prev and k <= kb
        # exactly the base detections whose larger lateral sigma is within the limit
        expect = {kk for kk, s in zip(zip(base["frame"].tolist(), base["row"].tolist(), base["col"].tolist()), sig)
                  if s <= lim}
        assert k == expect
        prev = k
    assert len(oracle.localize(frames, spec, w, max_sigma_px=0.5 * sig.min())) == 0
    assert keys(oracle.localize(frames, spec, w, max_sigma_px=2.0 * sig.max())) == kb
