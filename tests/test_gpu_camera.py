"""Per-pixel sCMOS camera maps (dl_set_camera_maps) on the GPU:

* constant maps equal to the config's scalars reproduce the scalar run bit for
  bit in every precision form (the same FP32 products);
* frames rendered through a seeded sCMOS sensor, with that sensor's maps set,
  match the FP64 oracle given the same maps (maps within 1e-4 relative,
  emitter sets equal outside the exempt pixels), on non-square and ragged
  frames, and differ from the scalar-path result;
* the tile gate's pooling reads the maps: its keep decisions equal the
  oracle gate's on pooled tiles preprocessed with the maps, and the handle's
  own pooling entry point (what gate training uses) matches the oracle's
  pooling with the scalars and then with the maps;
* frames of another shape and ROI lists are refused; graphs captured under
  another camera state refuse to launch, and graphs see new values of the
  same shape.
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
from tests.test_gpu_fp32 import TOL, gpu_localize, gpu_maps, make  # noqa: E402
from tests.test_gpu_gated import brightness_gate  # noqa: E402

DEV = torch.device("cuda:0")


@pytest.mark.parametrize("precision", ["fp32", "bf16", "fp8"])
def test_constant_maps_equal_scalar_path_bitwise(precision):
    spec, w, net = make("B", 2, precision=precision)
    frames = S.render_frames(2, 96, 160, "full", 71)
    m0 = gpu_maps(net, frames)
    r0, c0 = gpu_localize(net, frames)
    net.set_camera_maps(np.full((96, 160), 0.5, np.float32), np.full((96, 160), 100.0, np.float32))
    m1 = gpu_maps(net, frames)
    r1, c1 = gpu_localize(net, frames)
    assert np.array_equal(m0, m1) and np.array_equal(r0, r1) and np.array_equal(c0, c1)


@pytest.mark.parametrize("name,h,w", [("A", 200, 264), ("B", 136, 200), ("A", 77, 131)])
def test_scmos_frames_match_oracle(name, h, w):
    spec, wts, net = make(name, 1 if name == "A" else 2)
    cam = S.scmos_camera(h, w, 21)
    frames = S.render_frames(2, h, w, "tiny" if name == "A" else "full", 72, camera=cam)
    ref, ref_maps = oracle.localize(frames, spec, wts, gain=cam.gain, offset=cam.offset, return_maps=True)
    scalar = gpu_maps(net, frames)
    net.set_camera_maps(cam.gain, cam.offset)
    got = gpu_maps(net, frames)
    err = map_rel_err(got, ref_maps)
    print(name, h, w, "map rel err", err)
    assert err.max() <= TOL
    assert np.abs(got - scalar).max() > 1e-3                        # the maps matter
    rec, counts = gpu_localize(net, frames)
    cmp = compare_emitters(rec, ref, ref_maps)
    print(cmp)
    assert cmp["non_exempt_mismatch"] == 0 and cmp["order_ok"] and counts[-1] == len(rec)


def test_gate_pooling_reads_the_maps():
    h = w = 512
    cam = S.scmos_camera(h, w, 23, offset_sd=8.0)
    frames = S.render_frames(2, h, w, "sparse", 4044, camera=cam)
    pooled = []
    for F in frames:
        x = oracle.preprocess(F, cam.gain, cam.offset, 0.01)
        for ty in range(2):
            for tx in range(2):
                pooled.append(oracle.gate_pool(x[ty * 256:(ty + 1) * 256, tx * 256:(tx + 1) * 256], 4))
    pooled = np.stack(pooled)
    peaks = np.sort(np.maximum(pooled, 0).max(axis=(1, 2)))
    gaps = np.diff(peaks)
    mid = int(np.argmax(gaps))
    level = 0.5 * (peaks[mid] + peaks[mid + 1])
    th = brightness_gate(level)
    ref_keep = 1 / (1 + np.exp(-oracle.gate_forward(pooled, th))) > 0.05
    assert 0 < ref_keep.sum() < ref_keep.size
    spec, wts = S.make_net("A", 1)
    assert spec.in_scale == 0.01
    net = dl.Net(S.serialize_weights(spec, wts), flags=dl.DL_FLAG_GATE)
    net.set_gate(th.astype(np.float32), 0.05)
    net.set_camera_maps(cam.gain, cam.offset)
    gpu_localize(net, frames)
    k = torch.zeros(8, dtype=torch.uint8, device=DEV)
    net.gate_keep_map(k)
    torch.cuda.synchronize()
    assert np.array_equal(k.cpu().numpy().astype(bool), ref_keep)


def test_shape_mismatch_and_rois_are_refused():
    spec, w, net = make("A", 1)
    cam = S.scmos_camera(64, 80, 24)
    net.set_camera_maps(cam.gain, cam.offset)
    frames = S.render_frames(1, 64, 96, "tiny", 73)
    with pytest.raises(dl.DlocError) as e:
        gpu_maps(net, frames)
    assert e.value.code == dl.DL_ERR_INVALID_ARG
    roi = torch.from_numpy(S.render_frames(1, 64, 80, "tiny", 74)[0]).to(DEV)
    out = torch.zeros((256, 8), dtype=torch.int32, device=DEV)
    counts = torch.zeros(2, dtype=torch.int32, device=DEV)
    with pytest.raises(dl.DlocError) as e:
        net.localize_rois_device([roi], out, counts)
    assert e.value.code == dl.DL_ERR_UNSUPPORTED
    with pytest.raises(ValueError):
        net.set_camera_maps(cam.gain, cam.offset[:, :40])
    bad = cam.gain.copy()
    bad[3, 5] = 0.0
    with pytest.raises(dl.DlocError):
        net.set_camera_maps(bad, cam.offset)
    net.set_camera_maps(None, None)                  # cleared: any shape, ROIs again
    gpu_maps(net, frames)
    net.localize_rois_device([roi], out, counts)
    torch.cuda.synchronize()


def test_graphs_follow_the_camera_state():
    spec, w, net = make("A", 1)
    h, wd = 96, 128
    frames = S.render_frames(2, h, wd, "tiny", 75)
    fr = torch.from_numpy(frames).to(DEV)
    out = torch.zeros((4096, 8), dtype=torch.int32, device=DEV)
    counts = torch.zeros(3, dtype=torch.int32, device=DEV)
    g0 = net.graph(fr, out, counts)                  # captured with the scalars
    cam = S.scmos_camera(h, wd, 25, offset_sd=10.0)
    net.set_camera_maps(cam.gain, cam.offset)
    with pytest.raises(dl.DlocError) as e:
        g0.launch()
    assert e.value.code == dl.DL_ERR_INVALID_ARG
    g1 = net.graph(fr, out, counts)                  # captured with the maps
    cam2 = S.scmos_camera(h, wd, 26, offset_sd=10.0)
    net.set_camera_maps(cam2.gain, cam2.offset)      # same shape: updated in place
    ref, rc = gpu_localize(net, frames)
    for _ in range(3):
        counts.zero_()
        g1.launch()
        torch.cuda.synchronize()
        c = counts.cpu().numpy()
        assert np.array_equal(c, rc)
        assert np.array_equal(dl.emitters_from_device(out, int(c[-1])), ref)
    g0.close()
    g1.close()


def test_handle_gate_pool_uses_the_handle_preprocessing():
    """dl_gate_pool_net pools with the handle's scalars, or its camera maps once
    set: against the oracle's pooling of the preprocessed frames."""
    h, w = 256, 512
    cam = S.scmos_camera(h, w, 27, offset_sd=8.0)
    frames = S.render_frames(2, h, w, "sparse", 4045, camera=cam)
    spec, wts = S.make_net("A", 1)
    net = dl.Net(S.serialize_weights(spec, wts))
    fr = torch.from_numpy(frames).to(DEV)
    for maps in (False, True):
        if maps:
            net.set_camera_maps(cam.gain, cam.offset)
        p = torch.full((4, 64, 64), float("nan"), dtype=torch.float32, device=DEV)
        net.gate_pool(fr, p)
        torch.cuda.synchronize()
        got = p.cpu().numpy()
        ref = []
        for F in frames:
            x = oracle.preprocess(F, cam.gain if maps else 0.5, cam.offset if maps else 100.0, spec.in_scale)
            for tx in range(2):
                ref.append(oracle.gate_pool(x[:, tx * 256:(tx + 1) * 256], 4))
        ref = np.stack(ref)
        assert np.allclose(got, ref, rtol=1e-5, atol=1e-6 * np.abs(ref).max()), maps
    with pytest.raises(dl.DlocError) as e:
        net.gate_pool(fr[:, :, :256].contiguous(), torch.empty((2, 64, 64), dtype=torch.float32, device=DEV))
    assert e.value.code == dl.DL_ERR_INVALID_ARG      # not the sensor's shape


def test_host_entry_points_use_the_maps():
    """dl_localize and the pipelined host path with camera maps set give the
    device path's records (pageable frames, overlap on)."""
    spec, w, net = make("A", 1)
    h, wd = 96, 144
    cam = S.scmos_camera(h, wd, 28, offset_sd=10.0)
    net.set_camera_maps(cam.gain, cam.offset)
    frames = S.render_frames(4, h, wd, "tiny", 76, camera=cam)
    ref = []
    for k in range(2):
        r, _ = gpu_localize(net, frames[2 * k:2 * k + 2])
        r = r.copy()
        r["frame"] += 2 * k
        ref.append(r)
    ref = np.concatenate(ref)
    assert np.array_equal(net.localize(frames[:2]), ref[ref["frame"] < 2])
    assert np.array_equal(net.localize_pipelined(frames.reshape(2, 2, h, wd), overlap=True), ref)
