"""The 10-output head (per-pixel uncertainties of x, y, z and photons and the
background) on the GPU:

* FP32 maps, all ten planes, match the FP64 oracle within 1e-4 relative on
  ragged frames of nets A and B; emitter sets match outside the exempt pixels;
* each record's uncertainties are softplus of the GPU's own raw planes times
  their units (1e-6 relative), and agree with the oracle's records;
* the first five planes and the records equal those of the 5-output net with
  the same weights, in every precision form;
* dl_localize_device on the 10-output net gives the same records; the
  capacity limit cuts records and uncertainties alike; a 5-output net refuses
  dl_localize_device_unc;
* the uncertainty filter (max_sigma_px) keeps the oracle's filtered set;
* uneven ROI batches: ten maps per ROI against the oracle, records with
  uncertainties equal to the per-ROI runs; a graph of the 10-output net
  replays the eager records;
* a keep-all gate on sCMOS frames with camera maps gives the ungated records
  and uncertainties bit for bit;
* the host entry points return the device path's records and uncertainties.
"""
import numpy as np
import pytest

import oracle
import smlm_synth as S

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no HIP device", allow_module_level=True)
import paper_2410_02314_amd as dl  # noqa: E402
from tests.parity import compare_emitters, map_rel_err  # noqa: E402
from tests.test_gpu_fp32 import TOL, gpu_localize, gpu_maps  # noqa: E402

DEV = torch.device("cuda:0")


def make(name, precision="fp32"):
    spec, w = S.make_net(name, 1 if name[0] == "A" else 2)
    return spec, w, dl.Net(S.serialize_weights(spec, w), precision=precision)


def localize_unc(net, frames, cap=None):
    n, h, w = frames.shape
    fr = torch.from_numpy(np.ascontiguousarray(frames)).to(DEV)
    cap = cap if cap is not None else max(64, n * h * w // 8)
    out = torch.zeros((cap, 8), dtype=torch.int32, device=DEV)
    unc = torch.full((cap * 5,), float("nan"), dtype=torch.float32, device=DEV)
    counts = torch.full((n + 1,), -1, dtype=torch.int32, device=DEV)
    net.localize_device_unc(fr, out, unc, counts)
    torch.cuda.synchronize()
    c = counts.cpu().numpy().astype(np.int64)
    k = min(int(c[n]), cap)
    return dl.emitters_from_device(out, k), dl.uncertainties_from_device(unc, k), c


def softplus64(u):
    u = np.asarray(u, np.float64)
    return np.maximum(u, 0.0) + np.log1p(np.exp(-np.abs(u)))


@pytest.mark.parametrize("name,h,w", [("AU", 130, 200), ("BU", 96, 152)])
def test_fp32_maps_records_and_uncertainties_match_oracle(name, h, w):
    spec, wts, net = make(name)
    assert net.head_outputs == 10
    frames = S.render_frames(2, h, w, "tiny" if name == "AU" else "full", 81)
    ref, ref_unc, ref_maps = oracle.localize(frames, spec, wts, with_uncertainty=True, return_maps=True)
    got = gpu_maps(net, frames)
    assert got.shape == (2, 10, h, w)
    err = map_rel_err(got, ref_maps)
    print(name, "map rel err per plane", err)
    assert err.max() <= TOL
    rec, unc, counts = localize_unc(net, frames)
    cmp = compare_emitters(rec, ref, ref_maps)
    print(cmp)
    assert cmp["non_exempt_mismatch"] == 0 and cmp["order_ok"] and counts[-1] == len(rec) == len(unc)
    # each record's uncertainties from the GPU's own raw planes, in their units
    raw = got[rec["frame"], 5:, rec["row"], rec["col"]]          # [k][5]
    unit = np.array([1.0, 1.0, spec.z_scale, spec.ph_scale, 1.0 / spec.in_scale])
    floor = np.array([oracle.SIGMA_FLOOR] * 4 + [0.0])          # the sigmas' floor; none on the background
    expect = (softplus64(raw) + floor) * unit
    gotu = np.stack([unc[f] for f in unc.dtype.names], axis=1).astype(np.float64)
    assert np.all(gotu > 0)
    assert np.allclose(gotu, expect, rtol=1e-6, atol=0)
    # and against the oracle's records at the same pixels
    key = {(int(a), int(b), int(c)): i for i, (a, b, c) in enumerate(zip(ref["frame"], ref["row"], ref["col"]))}
    pairs = [(i, key[k]) for i, k in enumerate(zip(rec["frame"].tolist(), rec["row"].tolist(), rec["col"].tolist()))
             if k in key]
    assert len(pairs) >= 0.99 * len(rec)
    gi, ri = np.array([p[0] for p in pairs]), np.array([p[1] for p in pairs])
    refu = np.stack([ref_unc[f] for f in ref_unc.dtype.names], axis=1)[ri]
    assert np.allclose(gotu[gi], refu, rtol=1e-3, atol=1e-4 * unit)


@pytest.mark.parametrize("precision", ["fp32", "bf16", "fp8"])
def test_first_five_planes_and_records_equal_the_five_output_net(precision):
    s5, w5, n5 = make("B", precision)
    s10, w10, n10 = make("BU", precision)
    frames = S.render_frames(2, 112, 176, "full", 82)
    m5 = gpu_maps(n5, frames)
    m10 = gpu_maps(n10, frames)
    scale = np.abs(m5).max(axis=(0, 2, 3))
    assert np.all(np.abs(m10[:, :5] - m5).max(axis=(0, 2, 3)) <= 1e-6 * scale)
    assert np.all(np.isfinite(m10[:, 5:]))
    r5, c5 = gpu_localize(n5, frames)
    r10, u10, c10 = localize_unc(n10, frames)
    assert np.array_equal(r5, r10) and np.array_equal(c5, c10)
    assert np.all(np.stack([u10[f] for f in u10.dtype.names]) > 0)


def test_plain_entry_point_capacity_and_refusal():
    spec, w, net = make("AU")
    frames = S.render_frames(3, 128, 160, "tiny", 83)
    rec, unc, c = localize_unc(net, frames)
    plain, cp = gpu_localize(net, frames)
    assert np.array_equal(plain, rec) and np.array_equal(cp, c)
    k = len(rec) // 2
    assert k > 0
    rk, uk, ck = localize_unc(net, frames, cap=k)
    assert ck[-1] == len(rec) and len(rk) == k
    assert np.array_equal(rk, rec[:k]) and np.array_equal(uk, unc[:k])
    _, _, n5 = make("A")
    with pytest.raises(dl.DlocError) as e:
        localize_unc(n5, frames)
    assert e.value.code == dl.DL_ERR_UNSUPPORTED


def test_sigma_filter_matches_oracle():
    """max_sigma_px: the GPU keeps exactly the oracle's filtered detections,
    except pixels exempt under the usual threshold rules or whose sigma lies
    within 1e-4 (relative) of the limit; records and uncertainties stay
    aligned; a 5-output net refuses the setting."""
    from tests.parity import exempt_mask
    spec, wts = S.make_net("AU", 1)
    frames = S.render_frames(2, 128, 160, "tiny", 84)
    base, unc, maps = oracle.localize(frames, spec, wts, with_uncertainty=True, return_maps=True)
    sig = np.maximum(unc["sigma_x"], unc["sigma_y"])
    lim = float(np.median(sig))
    ref = oracle.localize(frames, spec, wts, max_sigma_px=lim)
    assert 0 < len(ref) < len(base)
    net = dl.Net(S.serialize_weights(spec, wts), max_sigma_px=lim)
    rec, u, counts = localize_unc(net, frames)
    keys = lambda r: set(zip(r["frame"].tolist(), r["row"].tolist(), r["col"].tolist()))  # noqa: E731
    base_keys = zip(base["frame"].tolist(), base["row"].tolist(), base["col"].tolist())
    near = {k for k, s in zip(base_keys, sig) if abs(s - lim) <= 1e-4 * lim}
    ex = [exempt_mask(maps[f, 0]) for f in range(len(frames))]
    diff = keys(rec) ^ keys(ref)
    bad = [k for k in diff if k not in near and not ex[k[0]][k[1], k[2]]]
    assert not bad, bad[:10]
    assert counts[-1] == len(rec) == len(u)
    assert np.all(np.maximum(u["sigma_x_px"], u["sigma_y_px"]) <= lim * (1 + 1e-4))
    plain, _ = gpu_localize(net, frames)
    assert np.array_equal(plain, rec)
    with pytest.raises(dl.DlocError) as e:
        make("A")[2].set_config(max_sigma_px=0.5)
    assert e.value.code == dl.DL_ERR_UNSUPPORTED


def test_uneven_rois_with_uncertainties():
    """ROI batches of a 10-output net: each ROI's ten maps against the oracle,
    and the ROI records with uncertainties equal the per-ROI device runs."""
    shapes = [(64, 96), (128, 64), (33, 200), (1, 130), (17, 5)]
    rois = S.render_rois(len(shapes), "rois", 1006, shapes=shapes)
    spec, wts, net = make("AU")
    d = [torch.from_numpy(r).to(DEV) for r in rois]
    px = sum(r.size for r in rois)
    maps = torch.full((10 * px,), float("nan"), dtype=torch.float32, device=DEV)
    net.maps_rois_device(d, maps)
    cap = 4096
    out = torch.zeros((cap, 8), dtype=torch.int32, device=DEV)
    unc = torch.zeros((cap * 5,), dtype=torch.float32, device=DEV)
    counts = torch.zeros(len(rois) + 1, dtype=torch.int32, device=DEV)
    net.localize_rois_device_unc(d, out, unc, counts)
    torch.cuda.synchronize()
    m, off = maps.cpu().numpy(), 0
    c = counts.cpu().numpy()
    rec = dl.emitters_from_device(out, int(c[-1]))
    u = dl.uncertainties_from_device(unc, int(c[-1]))
    for k, r in enumerate(rois):
        mk = m[off:off + 10 * r.size].reshape(10, *r.shape)
        off += 10 * r.size
        assert map_rel_err(mk, oracle.net_maps(r, spec, wts)).max() <= TOL, k
        rk, uk, _ = localize_unc(net, r[None])
        sel = rec["frame"] == k
        g = rec[sel].copy()
        g["frame"] = 0
        assert np.array_equal(g, rk) and np.array_equal(u[sel], uk), k


def test_graph_of_the_ten_output_net():
    spec, wts, net = make("AU")
    frames = S.render_frames(2, 96, 128, "tiny", 85)
    fr = torch.from_numpy(frames).to(DEV)
    out = torch.zeros((4096, 8), dtype=torch.int32, device=DEV)
    counts = torch.zeros(3, dtype=torch.int32, device=DEV)
    g = net.graph(fr, out, counts)
    ref, rc = gpu_localize(net, frames)
    for _ in range(3):
        counts.zero_()
        g.launch()
        torch.cuda.synchronize()
        c = counts.cpu().numpy()
        assert np.array_equal(c, rc) and np.array_equal(dl.emitters_from_device(out, int(c[-1])), ref)
    g.close()


def test_gate_camera_maps_and_uncertainties_together():
    """A gate that keeps every tile, on sCMOS frames with camera maps, through
    the 10-output head: records and uncertainties equal the ungated run bit for
    bit."""
    spec, wts = S.make_net("AU", 1)
    h = w = 512
    cam = S.scmos_camera(h, w, 29)
    frames = S.render_frames(2, h, w, "sparse", 4047, camera=cam)
    blob = S.serialize_weights(spec, wts)
    plain = dl.Net(blob)
    plain.set_camera_maps(cam.gain, cam.offset)
    r0, u0, c0 = localize_unc(plain, frames)
    gated = dl.Net(blob, flags=dl.DL_FLAG_GATE)
    gated.set_camera_maps(cam.gain, cam.offset)
    th = np.zeros(673, np.float32)
    th[672] = 20.0                                        # keeps every tile
    gated.set_gate(th, 0.05)
    r1, u1, c1 = localize_unc(gated, frames)
    assert len(r0) > 0
    assert np.array_equal(r0, r1) and np.array_equal(u0, u1) and np.array_equal(c0, c1)


@pytest.mark.parametrize("overlap", [True, False])
def test_host_entry_points_with_uncertainties(overlap):
    """dl_localize_unc and dl_localize_pipelined_unc give the device path's
    records and uncertainties (records of later batches counted across
    batches); a 5-output net refuses them."""
    spec, wts, net = make("AU")
    frames = S.render_frames(6, 96, 128, "tiny", 86).reshape(3, 2, 96, 128)
    ref_r, ref_u = [], []
    for k in range(3):
        r, u, _ = localize_unc(net, frames[k])
        r = r.copy()
        r["frame"] += 2 * k
        ref_r.append(r)
        ref_u.append(u)
    got_r, got_u = net.localize_pipelined_unc(frames, overlap=overlap)
    assert np.array_equal(got_r, np.concatenate(ref_r)) and np.array_equal(got_u, np.concatenate(ref_u))
    r1, u1 = net.localize_unc(frames[1])
    assert np.array_equal(u1, ref_u[1])
    _, _, n5 = make("A")
    with pytest.raises(dl.DlocError) as e:
        n5.localize_unc(frames[0])
    assert e.value.code == dl.DL_ERR_UNSUPPORTED
