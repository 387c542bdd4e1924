"""GPU parity of the dense-connection network (DLD1 blobs) against the FP64
oracle, through the C ABI.

The network (paper Sec. 3.2: every layer of a block reads the outputs of all
layers before it; Sec. 3.2.1 / Sec. 4.1.2: one dilation per block, 2, 4, 8,
16) runs in FP32 on MFMA: the bar is the FP32 path's, maps within 1e-4
relative (|g - o| <= 1e-4 (|o| + rms)), emitter sets identical except exempt
pixels (threshold band / near ties), integer work bit-exact.  Cases: net D
(C = 32, four blocks of four layers, growth 16) on tiny, ragged and
degenerate frames with random biases, a calibrated batch's emitters, full-size
2048^2 frames on sampled windows (margin: the receptive radius 121), ROI
lists and a capacity graph, the allocation-free entry point; a second layout
(C = 16, growth 32, three layers, 10 outputs) for the other kernel
instances; and the refusals of what the dense kernels do not support.

Net DU adds the two-stage U-Net after the blocks (Sec. 3.2: fine-grained
processing by a two-stage U-Net; its sizes are a reading): 2 x 2 max pooling,
3x3 convolutions at levels 1 and 2, nearest upsampling and 3x3 convolutions
over [skip, upsampled].  It is held to the same bar on odd-sized frames (edge
pooling windows hold fewer pixels), full-size windows (margin 133, crops
aligned to 4 pixels), ROI lists, fixed ROI graphs and the allocation-free
entry point.
"""
import numpy as np
import pytest

import oracle
import smlm_synth as S
from tests.parity import compare_emitters, exempt_mask, map_rel_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no HIP device", allow_module_level=True)
import paper_2410_02314_amd as dl  # noqa: E402

DEV = torch.device("cuda:0")
TOL = 1e-4
# C = 16, growth 32, 3 layers, dilations 1 and 3 (a dilation that is not a
# power of two), uncertainty head
NET_E = S.DenseSpec("E", 16, (1, 3), layers=3, growth=32, head_outputs=10)


def make(spec="D", seed=3, bias_std=0.0, **cfg):
    if isinstance(spec, str):
        spec, w = S.make_net(spec, seed, bias_std=bias_std)
    else:
        spec, w = S.make_net(spec, seed, calibrated=False, bias_std=bias_std)
    return spec, w, dl.Net(S.serialize_weights(spec, w), **cfg)


def gpu_maps(net, frames):
    n, h, w = frames.shape
    fr = torch.from_numpy(np.ascontiguousarray(frames)).to(DEV)
    maps = torch.full((n, net.head_outputs, h, w), float("nan"), dtype=torch.float32, device=DEV)
    net.maps_device(fr, maps)
    torch.cuda.synchronize()
    return maps.cpu().numpy()


def gpu_localize(net, frames, cap=None, noalloc=False):
    n, h, w = frames.shape
    fr = torch.from_numpy(np.ascontiguousarray(frames)).to(DEV)
    cap = cap if cap is not None else max(64, n * h * w // 2)   # local maxima: at most one pixel in two
    out = torch.zeros((cap, 8), dtype=torch.int32, device=DEV)
    counts = torch.full((n + 1,), -1, dtype=torch.int32, device=DEV)
    (net.localize_device_noalloc if noalloc else net.localize_device)(fr, out, counts)
    torch.cuda.synchronize()
    c = counts.cpu().numpy().astype(np.int64)
    return dl.emitters_from_device(out, min(int(c[n]), cap)), c


def test_inspect_dense_blob():
    spec, w = S.make_net("D", 3)
    info = dl.inspect_weights(S.serialize_weights(spec, w))
    assert info["C"] == 32 and info["dilations"] == (2, 4, 8, 16)
    assert info["dense_layers"] == 4 and info["dense_growth"] == 16
    assert info["receptive_radius"] == 121 and info["nparams"] == S.param_count(spec)


@pytest.mark.parametrize("spec,n,h,w", [("D", 2, 77, 131), ("D", 1, 40, 300), (NET_E, 2, 67, 90)])
def test_maps_ragged_frames_random_biases(spec, n, h, w):
    """Frames that are not multiples of the 8 x 32 tile at any dilation, random
    non-zero biases in every layer."""
    spec, wts, net = make(spec, 7, bias_std=0.05)
    frames = S.render_frames(n, h, w, "tiny", 555)
    ref = oracle.net_maps_batch(frames, spec, wts)
    got = gpu_maps(net, frames)
    assert not np.isnan(got).any()
    err = map_rel_err(got, ref)
    print(spec.name, (n, h, w), "map rel err", err.max())
    assert err.max() <= TOL


@pytest.mark.parametrize("h,w", [(1, 1), (1, 70), (5, 3), (9, 33), (2, 129)])
def test_tiny_and_degenerate_shapes(h, w):
    spec, wts, net = make("D", 4, bias_std=0.1)
    frames = S.render_frames(2, h, w, "tiny", 8)
    ref, ref_maps = oracle.localize(frames, spec, wts, return_maps=True)
    assert map_rel_err(gpu_maps(net, frames), ref_maps).max() <= TOL
    rec, counts = gpu_localize(net, frames)
    assert compare_emitters(rec, ref, ref_maps)["non_exempt_mismatch"] == 0 and counts[-1] == len(rec)


def test_calibrated_emitters_and_determinism():
    """Net D with its calibrated head on 2 x 256^2 full-model frames: the
    emitter set, per-frame counts and record order agree with the oracle; two
    runs give the same bits."""
    spec, wts, net = make("D", 3)
    frames = S.render_frames(2, 256, 256, "full", 1001)
    ref, ref_maps = oracle.localize(frames, spec, wts, return_maps=True)
    got = gpu_maps(net, frames)
    assert map_rel_err(got, ref_maps).max() <= TOL
    rec, counts = gpu_localize(net, frames)
    cmp = compare_emitters(rec, ref, ref_maps)
    print(cmp, len(ref))
    assert len(ref) > 30
    assert cmp["non_exempt_mismatch"] == 0 and cmp["order_ok"] and cmp["max_dxy_px"] < 1e-3
    assert list(counts[:2]) == list(np.bincount(rec["frame"], minlength=2)) and counts[2] == len(rec)
    rec2, counts2 = gpu_localize(net, frames)
    assert np.array_equal(rec, rec2) and np.array_equal(counts, counts2)
    assert np.array_equal(got, gpu_maps(net, frames))


def test_uncertainty_head_records():
    """The 10-output layout: records and their uncertainties match the oracle's."""
    spec, wts, net = make(NET_E, 9, bias_std=0.05)
    frames = S.render_frames(1, 96, 128, "tiny", 41)
    ref, ref_maps = oracle.localize(frames, spec, wts, return_maps=True)
    got = gpu_maps(net, frames)
    assert map_rel_err(got, ref_maps).max() <= TOL
    rec, _ = gpu_localize(net, frames)
    assert compare_emitters(rec, ref, ref_maps)["non_exempt_mismatch"] == 0


def test_full_size_sampled_windows():
    """2 x 2048^2 frames (the benchmark's frame size) on the GPU; the oracle
    computes sampled 40 x 48 windows exactly from a crop with the receptive
    radius (121 pixels) as margin."""
    spec, wts, net = make("D", 3)
    frames = S.render_frames(2, 2048, 2048, "full", 1002)
    got = gpu_maps(net, frames)
    rec, counts = gpu_localize(net, frames)
    assert counts[-1] == len(rec)
    for f, y0, x0 in [(0, 0, 0), (1, 1000, 517), (0, 2048 - 40, 2048 - 48)]:
        hh, ww = 40, 48
        print("window", f, y0, x0, flush=True)
        ref = oracle.net_maps_window(frames[f], spec, wts, y0, x0, hh, ww)
        err = map_rel_err(got[f, :, y0:y0 + hh, x0:x0 + ww], ref)
        assert err.max() <= TOL, (f, y0, x0, err.max())
        ref_det = oracle.detect(ref[0])[1:-1, 1:-1]
        ex = exempt_mask(ref[0])[1:-1, 1:-1]
        sel = ((rec["frame"] == f) & (rec["row"] > y0) & (rec["row"] < y0 + hh - 1) & (rec["col"] > x0)
               & (rec["col"] < x0 + ww - 1))
        gdet = np.zeros_like(ref_det)
        gdet[rec["row"][sel] - y0 - 1, rec["col"][sel] - x0 - 1] = True
        assert not np.any((gdet != ref_det) & ~ex)


def test_rois_and_capacity_graph():
    """An uneven ROI list (one a strided view): the eager ROI path agrees with
    the oracle per ROI; one capacity graph replayed over two ROI lists equals
    the eager path bit for bit."""
    spec, wts, net = make("D", 3)
    big = torch.from_numpy(S.render_frames(1, 200, 260, "rois", 95)[0]).to(DEV)
    sets = [[(64, 96), (33, 70), (1, 130), (90, 40)], [(48, 48)] * 3 + [(100, 120)]]
    cap_rois = 6
    out = torch.zeros((20000, 8), dtype=torch.int32, device=DEV)
    counts = torch.full((cap_rois + 1,), -1, dtype=torch.int32, device=DEV)
    g = net.graph_rois_dynamic(cap_rois, 200, 260, 60000, out, counts)
    for k, shapes in enumerate(sets):
        host = S.render_rois(len(shapes), "rois", 3000 + k, shapes=shapes)
        dev = [torch.from_numpy(np.ascontiguousarray(r)).to(DEV) for r in host]
        if k == 0:
            dev[0] = big[10:74, 20:116]
            host[0] = big[10:74, 20:116].cpu().numpy()
        e_out = torch.zeros((20000, 8), dtype=torch.int32, device=DEV)
        e_counts = torch.full((len(dev) + 1,), -1, dtype=torch.int32, device=DEV)
        net.localize_rois_device(dev, e_out, e_counts)
        torch.cuda.synchronize()
        ec = e_counts.cpu().numpy().astype(np.int64)
        erec = dl.emitters_from_device(e_out, int(ec[-1]))
        g.launch_rois(dev)
        torch.cuda.synchronize()
        c = counts.cpu().numpy()[:len(dev) + 1].astype(np.int64)
        assert np.array_equal(dl.emitters_from_device(out, int(c[-1])), erec) and np.array_equal(c, ec), k
        for j, r in enumerate(host):
            rr, mm = oracle.localize(np.ascontiguousarray(r)[None], spec, wts, return_maps=True)
            gj = erec[erec["frame"] == j].copy()
            gj["frame"] = 0
            cmp = compare_emitters(gj, rr, mm)
            assert cmp["non_exempt_mismatch"] == 0 and cmp["order_ok"], (k, j, cmp)
    g.close()


@pytest.mark.parametrize("queue", [1, 2])
def test_tile_queues_give_the_same_bits(queue):
    """The atomic tile queues (per XCD, global) only change which workgroup
    computes a tile: maps and records equal the static schedule's bit for bit,
    on a batch and on an uneven ROI list, twice in a row (the counters are
    cleared by every run)."""
    spec, wts, net = make("D", 3)
    _, _, netq = make("D", 3, tile_queue=queue)
    frames = S.render_frames(3, 200, 333, "full", 61)
    assert np.array_equal(gpu_maps(net, frames), gpu_maps(netq, frames))
    for _ in range(2):
        a, ca = gpu_localize(net, frames)
        b, cb = gpu_localize(netq, frames)
        assert np.array_equal(a, b) and np.array_equal(ca, cb)
    rois = [torch.from_numpy(r).to(DEV) for r in S.render_rois(5, "rois", 62, shapes=[(64, 90), (7, 300), (128, 128), (1, 1), (150, 40)])]
    outs = []
    for n_ in (net, netq):
        out = torch.zeros((20000, 8), dtype=torch.int32, device=DEV)
        counts = torch.full((6,), -1, dtype=torch.int32, device=DEV)
        n_.localize_rois_device(rois, out, counts)
        torch.cuda.synchronize()
        outs.append((dl.emitters_from_device(out, int(counts[-1].item())), counts.cpu().numpy()))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_noalloc_entry_point_matches():
    spec, wts, net = make("D", 3)
    for n, h, w in [(2, 128, 160), (1, 64, 64)]:
        frames = S.render_frames(n, h, w, "full", 77 + h)
        a, ca = gpu_localize(net, frames)
        b, cb = gpu_localize(net, frames, noalloc=True)
        assert np.array_equal(a, b) and np.array_equal(ca, cb)


def test_unsupported_settings_are_refused():
    spec, wts = S.make_net("D", 3)
    blob = S.serialize_weights(spec, wts)
    for cfg in ({"precision": "bf16"}, {"precision": "fp8"}, {"precision": "bf16x3"}, {"tile_rows": 4}):
        with pytest.raises(dl.DlocError) as e:
            dl.Net(blob, **cfg)
        assert e.value.code == dl.DL_ERR_UNSUPPORTED, cfg
    net = dl.Net(blob)
    with pytest.raises(dl.DlocError) as e:
        net.set_config(precision="bf16")
    assert e.value.code == dl.DL_ERR_UNSUPPORTED
    cam = S.scmos_camera(64, 64, 5)
    with pytest.raises(dl.DlocError) as e:
        net.set_camera_maps(cam.gain, cam.offset)
    assert e.value.code == dl.DL_ERR_UNSUPPORTED
    fr = torch.from_numpy(S.render_frames(1, 64, 64, "tiny", 3)).to(DEV)
    with pytest.raises(dl.DlocError) as e:
        net.autotune_ex(fr, reps=1)
    assert e.value.code == dl.DL_ERR_UNSUPPORTED
    # the handle still runs
    frames = S.render_frames(1, 64, 64, "tiny", 3)
    ref, ref_maps = oracle.localize(frames, spec, wts, return_maps=True)
    rec, _ = gpu_localize(net, frames)
    assert compare_emitters(rec, ref, ref_maps)["non_exempt_mismatch"] == 0


UNET_E = S.DenseSpec("UE", 16, (1, 3), layers=2, growth=32, unet=2, head_outputs=10)


def test_inspect_unet_blob():
    spec, w = S.make_net("DU", 3)
    info = dl.inspect_weights(S.serialize_weights(spec, w))
    assert info["unet_levels"] == 2 and info["receptive_radius"] == 133 == S.receptive_radius(spec)
    assert info["nparams"] == S.param_count(spec)
    assert dl.inspect_weights(S.serialize_weights(*S.make_net("D", 3)))["unet_levels"] == 0


@pytest.mark.parametrize("spec,n,h,w", [("DU", 2, 77, 131), ("DU", 1, 5, 3), ("DU", 2, 1, 1), ("DU", 1, 2, 129),
                                        (UNET_E, 2, 67, 90)])
def test_unet_maps_odd_frames_random_biases(spec, n, h, w):
    """Frames whose sides are odd at some level, so edge pooling windows hold
    fewer pixels, random biases everywhere."""
    spec, wts, net = make(spec, 7, bias_std=0.05)
    frames = S.render_frames(n, h, w, "tiny", 556)
    ref = oracle.net_maps_batch(frames, spec, wts)
    got = gpu_maps(net, frames)
    assert not np.isnan(got).any()
    err = map_rel_err(got, ref)
    print(spec.name, (n, h, w), "map rel err", err.max())
    assert err.max() <= TOL
    rec, counts = gpu_localize(net, frames)
    ref_rec = oracle.localize(frames, spec, wts)
    assert compare_emitters(rec, ref_rec, ref)["non_exempt_mismatch"] == 0 and counts[-1] == len(rec)


def test_unet_calibrated_emitters():
    spec, wts, net = make("DU", 3)
    frames = S.render_frames(2, 256, 256, "full", 1001)
    ref, ref_maps = oracle.localize(frames, spec, wts, return_maps=True)
    assert map_rel_err(gpu_maps(net, frames), ref_maps).max() <= TOL
    rec, counts = gpu_localize(net, frames)
    cmp = compare_emitters(rec, ref, ref_maps)
    print(cmp)
    assert len(ref) > 10 and cmp["non_exempt_mismatch"] == 0 and cmp["order_ok"] and cmp["max_dxy_px"] < 1e-3
    rec2, _ = gpu_localize(net, frames)
    assert np.array_equal(rec, rec2)


def test_unet_full_size_sampled_windows():
    spec, wts, net = make("DU", 3)
    frames = S.render_frames(1, 2048, 2048, "full", 1003)
    got = gpu_maps(net, frames)
    for y0, x0 in [(0, 0), (1001, 517), (2048 - 40, 2048 - 48)]:
        ref = oracle.net_maps_window(frames[0], spec, wts, y0, x0, 40, 48)
        err = map_rel_err(got[0, :, y0:y0 + 40, x0:x0 + 48], ref)
        print("window", y0, x0, err.max(), flush=True)
        assert err.max() <= TOL


def test_unet_rois_graph_and_noalloc():
    """ROI lists (one a strided view) against the oracle per ROI; a fixed ROI
    graph replays the eager records; the allocation-free entry point equals
    the allocating one; a capacity graph is refused."""
    spec, wts, net = make("DU", 3)
    big = torch.from_numpy(S.render_frames(1, 200, 260, "rois", 96)[0]).to(DEV)
    host = S.render_rois(4, "rois", 3100, shapes=[(64, 96), (33, 70), (1, 130), (90, 41)])
    dev = [torch.from_numpy(np.ascontiguousarray(r)).to(DEV) for r in host]
    dev[0] = big[11:75, 21:117]
    host[0] = big[11:75, 21:117].cpu().numpy()
    out = torch.zeros((20000, 8), dtype=torch.int32, device=DEV)
    counts = torch.full((5,), -1, dtype=torch.int32, device=DEV)
    net.localize_rois_device(dev, out, counts)
    torch.cuda.synchronize()
    c = counts.cpu().numpy().astype(np.int64)
    erec = dl.emitters_from_device(out, int(c[-1]))
    for j, r in enumerate(host):
        rr, mm = oracle.localize(np.ascontiguousarray(r)[None], spec, wts, return_maps=True)
        gj = erec[erec["frame"] == j].copy()
        gj["frame"] = 0
        assert compare_emitters(gj, rr, mm)["non_exempt_mismatch"] == 0, j
    g = net.graph_rois(dev, out, counts)
    for _ in range(2):
        out.zero_()
        g.launch()
        torch.cuda.synchronize()
        assert np.array_equal(dl.emitters_from_device(out, int(c[-1])), erec)
    g.close()
    with pytest.raises(dl.DlocError) as e:
        net.graph_rois_dynamic(4, 100, 130, 20000, out, counts)
    assert e.value.code == dl.DL_ERR_UNSUPPORTED
    for n, h, w in [(2, 96, 130), (1, 33, 33)]:
        frames = S.render_frames(n, h, w, "full", 90 + h)
        a, ca = gpu_localize(net, frames)
        b, cb = gpu_localize(net, frames, noalloc=True)
        assert np.array_equal(a, b) and np.array_equal(ca, cb)
