"""The boundary calls beyond the device-resident path, against the oracle:

* dl_localize_rois: uneven ROIs in host memory (some strided views of a larger
  frame) -> the oracle's records per ROI, and the device ROI path's records
  bit for bit;
* dl_localize_maps: host frames -> host maps, equal to dl_maps_device bit for
  bit and to the oracle within the FP32 tolerance;
* dl_debug_compact: the compaction step alone on given flags and maps -> the
  oracle's records (positions exact, values within FP32 rounding), capacity
  cut, empty frames;
* dl_config.in_scale_override: the same maps as weights carrying that
  in_scale, bit for bit, and the oracle's; tile_w accepts the form's width.
"""
import numpy as np
import pytest

import oracle
import smlm_synth as S
from tests.parity import compare_emitters, map_rel_err, record_field_errors

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no HIP device", allow_module_level=True)
import paper_2410_02314_amd as dl  # noqa: E402
from tests.test_gpu_fp32 import gpu_maps  # noqa: E402

DEV = torch.device("cuda:0")


def test_host_rois_match_oracle_and_device_path():
    spec, w = S.make_net("A", 1)
    net = dl.Net(S.serialize_weights(spec, w))
    shapes = [(64, 96), (33, 200), (1, 130), (120, 77), (17, 5)]
    rois = list(S.render_rois(len(shapes), "rois", 1004, shapes=shapes))
    big = S.render_frames(1, 150, 260, "tiny", 91)[0]
    rois += [big[10:74, 20:120], big[80:150, 150:260]]            # strided host views
    rec = net.localize_rois(rois)
    refs, maps = [], []
    for k, r in enumerate(rois):
        rr, mm = oracle.localize(np.ascontiguousarray(r)[None], spec, w, return_maps=True)
        rr["frame"] = k
        refs.append(rr)
        maps.append(mm[0])
    ref = np.concatenate(refs)
    for k in range(len(rois)):
        g = rec[rec["frame"] == k].copy()
        rk = ref[ref["frame"] == k].copy()
        g["frame"] = 0
        rk["frame"] = 0
        cmp = compare_emitters(g, rk, maps[k][None])
        assert cmp["non_exempt_mismatch"] == 0 and cmp["order_ok"], (k, cmp)
        err = record_field_errors(g, rk, maps[k][None], spec)
        assert max(err[f] for f in ("x", "y", "z", "photons", "prob")) <= 1.0, (k, err)
    # the device ROI path on the same pixels gives the same records
    dev = [torch.from_numpy(np.ascontiguousarray(r)).to(DEV) for r in rois]
    out = torch.zeros((4096, 8), dtype=torch.int32, device=DEV)
    counts = torch.zeros(len(rois) + 1, dtype=torch.int32, device=DEV)
    net.localize_rois_device(dev, out, counts)
    torch.cuda.synchronize()
    assert np.array_equal(dl.emitters_from_device(out, int(counts[-1].item())), rec)
    # capacity: the two-call protocol
    few = net.localize_rois(rois, cap=3)
    assert np.array_equal(few, rec)


def test_host_maps_equal_device_maps_and_oracle():
    spec, w = S.make_net("B", 2)
    net = dl.Net(S.serialize_weights(spec, w))
    frames = S.render_frames(2, 96, 140, "full", 92)
    got = net.localize_maps(frames)
    assert np.array_equal(got, gpu_maps(net, frames))
    ref = oracle.net_maps_batch(frames, spec, w)
    assert map_rel_err(got, ref).max() <= 1e-4


@pytest.mark.parametrize("nh", [5, 10])
def test_debug_compact_matches_oracle_records(nh):
    spec, w = S.make_net("A" if nh == 5 else "AU", 1)
    net = dl.Net(S.serialize_weights(spec, w))
    r = np.random.default_rng(9)
    n, h, wd = 3, 37, 150
    det = (r.random((n, h, wd)) < 0.05).astype(np.uint8)
    det[1] = 0                                          # a frame with nothing
    det[2, 0, :] = 1                                    # a full row
    maps = r.standard_normal((n, nh, h, wd)).astype(np.float32)
    cap = int(det.sum()) + 5
    out = torch.zeros((cap, 8), dtype=torch.int32, device=DEV)
    counts = torch.full((n + 1,), -1, dtype=torch.int32, device=DEV)
    net.debug_compact(torch.from_numpy(det).to(DEV), torch.from_numpy(maps).to(DEV), out, counts)
    torch.cuda.synchronize()
    c = counts.cpu().numpy()
    assert list(c[:n]) == [int(det[f].sum()) for f in range(n)] and c[n] == det.sum()
    got = dl.emitters_from_device(out, int(c[n]))
    ref = np.concatenate([oracle.records(maps[f].astype(np.float64), det[f].astype(bool), spec, f) for f in range(n)])
    assert np.array_equal(got["frame"], ref["frame"]) and np.array_equal(got["row"], ref["row"])
    assert np.array_equal(got["col"], ref["col"])
    for g_name, o_name in (("x_px", "x"), ("y_px", "y"), ("z_nm", "z"), ("photons", "photons"), ("prob", "prob")):
        assert np.allclose(got[g_name], ref[o_name], rtol=2e-7, atol=1e-6 * (1 + np.abs(ref[o_name]).max())), g_name
    # capacity cut: the first records, the totals unchanged
    small = torch.zeros((4, 8), dtype=torch.int32, device=DEV)
    net.debug_compact(torch.from_numpy(det).to(DEV), torch.from_numpy(maps).to(DEV), small, counts)
    torch.cuda.synchronize()
    assert int(counts[n].item()) == det.sum()
    assert np.array_equal(dl.emitters_from_device(small, 4), got[:4])


def test_in_scale_override_and_tile_w():
    spec, w = S.make_net("A", 1)
    frames = S.render_frames(2, 80, 96, "tiny", 93)
    base = dl.Net(S.serialize_weights(spec, w), in_scale_override=0.02)
    spec2 = S.NetSpec("A", spec.C, spec.dilations, in_scale=0.02)
    other = dl.Net(S.serialize_weights(spec2, w))
    got = gpu_maps(base, frames)
    assert np.array_equal(got, gpu_maps(other, frames))
    assert map_rel_err(got, oracle.net_maps_batch(frames, spec2, w)).max() <= 1e-4
    assert not np.array_equal(got, gpu_maps(dl.Net(S.serialize_weights(spec, w)), frames))
    # tile_w: the form's own width runs, others are refused
    same = dl.Net(S.serialize_weights(spec, w), tile_w=32)
    assert np.array_equal(gpu_maps(same, frames), gpu_maps(dl.Net(S.serialize_weights(spec, w)), frames))
    with pytest.raises(dl.DlocError) as e:
        dl.Net(S.serialize_weights(spec, w), tile_w=48)
    assert e.value.code == dl.DL_ERR_UNSUPPORTED
