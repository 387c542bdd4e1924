"""The learned tile gate, trained on the GPU by the library's own kernels, and
what it gains over running the network without it.

Training tiles come from sparse frames seeded apart from the evaluation frames
and are labelled by the ungated BF16 network's own detections.  The gate's
threshold is chosen on held-out training tiles to keep 99.9 % of their
detections (a margin over the 99.5 % recall target: the held-out set is small); on the evaluation frames the gate must then skip a substantial
share of the tiles while keeping nearly every ungated detection.  The
threshold for 99.5 % of the positive tiles, the fixed 0.05, the untrained
initial gate and a non-learned brightness rule (brightest pooled pixel above a
level chosen for the same 99.9 % of held-out detections) are reported beside
it.
"""
import numpy as np
import pytest

import smlm_synth as S

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no HIP device", allow_module_level=True)
import paper_2410_02314_amd as dl  # noqa: E402
from paper_2410_02314_amd import gate_train as GT  # noqa: E402
from tests.test_gpu_fp32 import gpu_localize  # noqa: E402

DEV = torch.device("cuda:0")
SIDE = 1024


def gated_eval(blob, theta, frames, thr):
    net = dl.Net(blob, precision="bf16", flags=dl.DL_FLAG_GATE)
    net.set_gate(theta, thr)
    rec, _ = gpu_localize(net, frames)
    k = torch.zeros(len(frames) * (SIDE // 256) ** 2, dtype=torch.uint8, device=DEV)
    net.gate_keep_map(k)
    torch.cuda.synchronize()
    return rec, k.cpu().numpy().astype(bool)


def test_trained_gate_skips_empty_tiles_and_keeps_detections():
    spec, w = S.make_net("B", 2)
    blob = S.serialize_weights(spec, w)
    net = dl.Net(blob, precision="bf16")
    batches = (S.render_frames(16, SIDE, SIDE, "sparse", 2005, frame_ids=range(k, k + 16)) for k in range(0, 160, 16))
    pooled, labels, counts = GT.labelled_tiles(net, batches, DEV, with_counts=True)
    assert pooled.shape[0] == 160 * 16
    frac_pos = float(labels.mean())
    theta0 = S.gate_flat(S.gate_init(3005))
    res = GT.train(pooled, labels, theta0, epochs=60, batch=256, lr=1e-2)
    hist = res.history
    print("positive tile fraction", frac_pos)
    print("first/last epoch", hist[0], hist[-1])
    assert hist[-1]["val_loss"] < hist[0]["val_loss"]

    ev = S.render_frames(16, SIDE, SIDE, "sparse", 1005)
    rec0, _ = gpu_localize(net, ev)
    ref = {(a, b, c) for a, b, c in zip(rec0["frame"], rec0["row"], rec0["col"])}
    out = {}
    thr = GT.threshold_at_recall(pooled, labels, res.theta, res.val_idx, 0.999, counts)
    # non-learned control: keep a tile if its brightest pooled pixel exceeds a
    # level chosen on the same held-out tiles for the same 99.9 % of detections
    from tests.test_gpu_gated import brightness_gate
    vi = np.asarray(res.val_idx)
    peak = np.maximum(pooled.cpu().numpy(), 0).max(axis=(1, 2))
    level = GT.threshold_for_recall(peak[vi], labels.cpu().numpy()[vi] > 0.5, 0.999, counts[vi])
    bright = brightness_gate(level).astype(np.float32)
    thr_tile = GT.threshold_at_recall(pooled, labels, res.theta, res.val_idx, 0.995)
    print("thresholds at 99.9% held-out detection / 99.5% tile recall:", thr, thr_tile)
    for name, th, p in [("trained", res.theta, thr), ("trained@tile-recall", res.theta, thr_tile),
                        ("trained@0.05", res.theta, 0.05), ("untrained@0.05", theta0, 0.05),
                        ("brightness", bright, 0.05)]:
        rec, keep = gated_eval(blob, th, ev, p)
        got = {(a, b, c) for a, b, c in zip(rec["frame"], rec["row"], rec["col"])}
        out[name] = {"threshold": p, "skip": float(1 - keep.mean()),
                     "recall_vs_ungated": len(got & ref) / max(1, len(ref)), "extra": len(got - ref)}
    print(out)
    t = out["trained"]
    assert t["recall_vs_ungated"] >= 0.99
    assert t["skip"] >= 0.2
    # at the fixed 0.05 the trained gate skips empty tiles with nearly full recall
    t5 = out["trained@0.05"]
    assert t5["skip"] >= 0.2 and t5["recall_vs_ungated"] >= 0.995
