"""Uneven batches: ROIs of different shapes (and strided ROIs cut out of a
larger frame) in one call, against the FP64 oracle per ROI."""
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
from tests.test_gpu_fp32 import gpu_localize, gpu_maps  # noqa: E402

DEV = torch.device("cuda:0")


def roi_run(net, rois_np, strided_from=None):
    """rois_np: list of uint16 arrays; returns (list of maps [5][h][w], records, counts)."""
    if strided_from is None:
        d = [torch.from_numpy(np.ascontiguousarray(r)).to(DEV) for r in rois_np]
    else:
        d = strided_from
    total = sum(r.shape[0] * r.shape[1] for r in rois_np)
    maps = torch.full((5 * total,), float("nan"), dtype=torch.float32, device=DEV)
    net.maps_rois_device(d, maps)
    cap = max(256, total // 8)
    out = torch.zeros((cap, 8), dtype=torch.int32, device=DEV)
    counts = torch.full((len(d) + 1,), -1, dtype=torch.int32, device=DEV)
    net.localize_rois_device(d, out, counts)
    torch.cuda.synchronize()
    m = maps.cpu().numpy()
    per, o = [], 0
    for r in rois_np:
        h, w = r.shape
        per.append(m[o:o + 5 * h * w].reshape(5, h, w))
        o += 5 * h * w
    c = counts.cpu().numpy().astype(np.int64)
    return per, dl.emitters_from_device(out, int(c[-1])), c


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_uneven_rois_match_oracle(prec):
    shapes = [(64, 96), (128, 64), (33, 200), (96, 96), (1, 130), (200, 37), (64, 64), (17, 5)]
    rois = S.render_rois(len(shapes), "rois", 1004, shapes=shapes)
    spec, w = S.make_net("A", 1)
    net = dl.Net(S.serialize_weights(spec, w), precision=prec)
    maps, rec, counts = roi_run(net, rois)
    quant = "exact" if prec == "fp32" else "bf16"
    refs, ref_maps = [], []
    for k, r in enumerate(rois):
        rr, mm = oracle.localize(r[None], spec, w, return_maps=True, quant="exact")
        rr["frame"] = k
        refs.append(rr)
        ref_maps.append(mm[0])
        if prec == "fp32":
            assert map_rel_err(maps[k], mm[0]).max() <= 1e-4, k
        else:
            emu = oracle.net_maps(r, spec, w, quant="bf16")
            assert np.all(map_rel_err(maps[k], emu) <= 2.0 * map_rel_err(emu, mm[0]) + 1e-4), k
    ref = np.concatenate(refs)
    assert counts[-1] == len(rec) and list(counts[:-1]) == list(np.bincount(rec["frame"], minlength=len(rois)))
    keys = list(zip(rec["frame"], rec["row"], rec["col"]))
    assert keys == sorted(keys)
    if prec == "fp32":
        for k in range(len(rois)):
            g = rec[rec["frame"] == k]
            g = g.copy()
            g["frame"] = 0
            rk = ref[ref["frame"] == k].copy()
            rk["frame"] = 0
            cmp = compare_emitters(g, rk, ref_maps[k][None])
            assert cmp["non_exempt_mismatch"] == 0, (k, cmp)


def test_strided_rois_cut_from_a_frame():
    big = S.render_frames(1, 300, 400, "tiny", 7)[0]
    d_big = torch.from_numpy(big).to(DEV)
    boxes = [(0, 0, 100, 128), (50, 70, 64, 200), (200, 10, 100, 390)]
    views = [d_big[y:y + h, x:x + w] for (y, x, h, w) in boxes]
    assert all(v.stride(0) == 400 for v in views)
    crops = [big[y:y + h, x:x + w] for (y, x, h, w) in boxes]
    spec, w = S.make_net("A", 1)
    net = dl.Net(S.serialize_weights(spec, w))
    maps, rec, counts = roi_run(net, crops, strided_from=views)
    for k, c in enumerate(crops):
        assert map_rel_err(maps[k], oracle.net_maps(c, spec, w)).max() <= 1e-4


def test_equal_rois_equal_uniform_batch_bitwise():
    frames = S.render_frames(3, 96, 160, "tiny", 12)
    spec, w = S.make_net("B", 2)
    net = dl.Net(S.serialize_weights(spec, w))
    maps, rec, counts = roi_run(net, list(frames))
    um = gpu_maps(net, frames)
    ur, uc = gpu_localize(net, frames)
    assert all(np.array_equal(maps[k], um[k]) for k in range(3))
    assert np.array_equal(rec, ur) and np.array_equal(counts, uc)


def test_full_roi_workload_sampled():
    """256 ROIs with sides from {128, ..., 1024} (the uneven-batch workload),
    checked against the oracle on a sample of ROIs computed whole."""
    rois = S.render_rois(256, "rois", 1004)
    spec, w = S.make_net("A", 1)
    net = dl.Net(S.serialize_weights(spec, w))
    maps, rec, counts = roi_run(net, rois)
    assert counts[-1] == len(rec)
    small = [k for k, r in enumerate(rois) if r.shape[0] * r.shape[1] <= 128 * 256][:4]
    for k in small:
        rr, mm = oracle.localize(rois[k][None], spec, w, return_maps=True)
        assert map_rel_err(maps[k], mm[0]).max() <= 1e-4
        g = rec[rec["frame"] == k].copy()
        g["frame"] = 0
        assert compare_emitters(g, rr, mm)["non_exempt_mismatch"] == 0
    # a window inside a large ROI
    big = max(range(256), key=lambda k: rois[k].size)
    H, W = rois[big].shape
    ref = oracle.net_maps_window(rois[big], spec, w, H // 2, W // 3, 24, 40)
    assert map_rel_err(maps[big][:, H // 2:H // 2 + 24, W // 3:W // 3 + 40], ref).max() <= 1e-4
