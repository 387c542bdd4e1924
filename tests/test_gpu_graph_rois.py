"""One graph, any ROI batch: dl_graph_create_rois_dynamic captures the path
once for a capacity; each replay takes a new ROI list (a pinned slot copied
by the graph, descriptors built on the device).  Replays over different ROI
sets -- different counts, shapes and strided views, in FP32 and BF16 -- equal
the eager ROI path bit for bit and the oracle per ROI; eager work between
replays does not disturb them; ROI lists past the capacity are refused."""
import numpy as np
import pytest

import oracle
import smlm_synth as S
from tests.parity import compare_emitters

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no HIP device", allow_module_level=True)
import paper_2410_02314_amd as dl  # noqa: E402

DEV = torch.device("cuda:0")


def eager(net, dev_rois, cap=20000):
    out = torch.zeros((cap, 8), dtype=torch.int32, device=DEV)
    counts = torch.full((len(dev_rois) + 1,), -1, dtype=torch.int32, device=DEV)
    net.localize_rois_device(dev_rois, out, counts)
    torch.cuda.synchronize()
    c = counts.cpu().numpy()
    return dl.emitters_from_device(out, int(c[-1])), c


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_one_graph_serves_different_roi_sets(prec):
    spec, w = S.make_net("A", 1)
    net = dl.Net(S.serialize_weights(spec, w), precision=prec)
    big = torch.from_numpy(S.render_frames(1, 300, 400, "rois", 95)[0]).to(DEV)
    sets = [
        [(64, 96), (128, 64), (33, 200), (1, 130), (200, 37)],
        [(256, 256), (17, 5), (90, 300)],
        [(40, 40)] * 9,
    ]
    cap_rois, cap_h, cap_w, cap_px = 12, 300, 400, 200000
    out = torch.zeros((20000, 8), dtype=torch.int32, device=DEV)
    counts = torch.full((cap_rois + 1,), -1, dtype=torch.int32, device=DEV)
    g = net.graph_rois_dynamic(cap_rois, cap_h, cap_w, cap_px, out, counts)
    print(f"graph {prec}: captured", flush=True)
    for k, shapes in enumerate(sets * 2):
        host = S.render_rois(len(shapes), "rois", 2000 + k % len(sets), shapes=shapes)
        dev = [torch.from_numpy(np.ascontiguousarray(r)).to(DEV) for r in host]
        if k == 1:                                          # strided views of a larger frame
            dev[0] = big[10:266, 20:276]
            host[0] = big[10:266, 20:276].cpu().numpy()
        torch.cuda.synchronize()
        g.launch_rois(dev)
        torch.cuda.synchronize()
        c = counts.cpu().numpy()[:len(dev) + 1].astype(np.int64)
        rec = dl.emitters_from_device(out, int(c[-1]))
        ref_rec, ref_c = eager(net, dev)                    # eager work between replays
        assert np.array_equal(rec, ref_rec) and np.array_equal(c, ref_c), k
        if prec == "fp32" and k < len(sets):
            for j, r in enumerate(host):
                rr, mm = oracle.localize(np.ascontiguousarray(r)[None], spec, w, return_maps=True)
                gj = rec[rec["frame"] == j].copy()
                gj["frame"] = 0
                cmp = compare_emitters(gj, rr, mm)
                assert cmp["non_exempt_mismatch"] == 0 and cmp["order_ok"], (k, j, cmp)
    g.close()


def test_roi_lists_past_the_capacity_are_refused():
    spec, w = S.make_net("A", 1)
    net = dl.Net(S.serialize_weights(spec, w))
    out = torch.zeros((1000, 8), dtype=torch.int32, device=DEV)
    counts = torch.zeros(5, dtype=torch.int32, device=DEV)
    g = net.graph_rois_dynamic(4, 100, 100, 20000, out, counts)
    frames = [torch.zeros((50, 50), dtype=torch.uint16, device=DEV) for _ in range(5)]
    for bad in (frames, [torch.zeros((101, 10), dtype=torch.uint16, device=DEV)],
                [torch.zeros((100, 100), dtype=torch.uint16, device=DEV)] * 3):
        with pytest.raises(dl.DlocError) as e:
            g.launch_rois(bad)
        assert e.value.code == dl.DL_ERR_CAPACITY
    with pytest.raises(dl.DlocError):
        g.launch(None)                                      # a capacity graph needs its ROI list
    g.launch_rois(frames[:2])                               # and still serves lists that fit
    torch.cuda.synchronize()
    c = counts.cpu().numpy()[:3].astype(np.int64)
    ref_rec, ref_c = eager(net, frames[:2])
    assert np.array_equal(c, ref_c) and np.array_equal(dl.emitters_from_device(out, int(c[-1])), ref_rec)
    g.close()
