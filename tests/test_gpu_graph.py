"""HIP-graph replay of the whole localization equals eager execution, replay
after replay, with the frame buffer refilled in place and eager work in
between (no memset nodes are captured; counters are cleared by kernels)."""
import numpy as np
import pytest

import smlm_synth as S

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no HIP device", allow_module_level=True)
import paper_2410_02314_amd as dl  # noqa: E402

DEV = torch.device("cuda:0")


def eager(net, d_frames, cap):
    out = torch.zeros((cap, 8), dtype=torch.int32, device=DEV)
    counts = torch.zeros(d_frames.shape[0] + 1, dtype=torch.int32, device=DEV)
    net.localize_device(d_frames, out, counts)
    torch.cuda.synchronize()
    n = int(counts[-1].item())
    return out[:n].clone(), counts.clone()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_graph_replays_match_eager(prec):
    spec, w = S.make_net("A", 1)
    net = dl.Net(S.serialize_weights(spec, w), precision=prec)
    batches = [S.render_frames(4, 128, 128, "tiny", s) for s in (1001, 1002, 1003)]
    buf = torch.from_numpy(batches[0]).to(DEV)
    cap = 4096
    out = torch.zeros((cap, 8), dtype=torch.int32, device=DEV)
    counts = torch.zeros(5, dtype=torch.int32, device=DEV)
    g = net.graph(buf, out, counts)
    for rep in range(6):
        frames = batches[rep % 3]
        buf.copy_(torch.from_numpy(frames).to(DEV))
        out.zero_()
        g.launch()
        torch.cuda.synchronize()
        n = int(counts[-1].item())
        got_out, got_counts = out[:n].clone(), counts.clone()
        ref_out, ref_counts = eager(net, torch.from_numpy(frames).to(DEV), cap)   # eager work between replays
        assert torch.equal(got_counts, ref_counts), rep
        assert torch.equal(got_out, ref_out), rep
    g.close()


def test_graph_rois_match_eager():
    shapes = [(128, 256), (384, 128), (64, 64), (256, 512)]
    rois = S.render_rois(len(shapes), "rois", 1004, shapes=shapes)
    spec, w = S.make_net("A", 1)
    net = dl.Net(S.serialize_weights(spec, w))
    d = [torch.from_numpy(r).to(DEV) for r in rois]
    cap = 1 << 15
    out = torch.zeros((cap, 8), dtype=torch.int32, device=DEV)
    counts = torch.zeros(len(d) + 1, dtype=torch.int32, device=DEV)
    g = net.graph_rois(d, out, counts)
    for rep in range(3):
        out.zero_()
        g.launch()
        torch.cuda.synchronize()
        n = int(counts[-1].item())
        got = out[:n].clone()
        out2 = torch.zeros((cap, 8), dtype=torch.int32, device=DEV)
        c2 = torch.zeros(len(d) + 1, dtype=torch.int32, device=DEV)
        net.localize_rois_device(d, out2, c2)
        torch.cuda.synchronize()
        assert torch.equal(c2, counts) and torch.equal(out2[:n], got)
    g.close()


def test_autotune_picks_a_candidate_and_keeps_results():
    spec, w = S.make_net("B", 2)
    net = dl.Net(S.serialize_weights(spec, w))
    frames = S.render_frames(2, 256, 384, "full", 5)
    d = torch.from_numpy(frames).to(DEV)
    ref, _ = eager(net, d, 1 << 14)
    rows, ms = net.autotune(d, reps=2)
    assert rows in (4, 8) and all(v > 0 for v in ms.values())
    assert ms[rows] == min(ms.values())
    got, _ = eager(net, d, 1 << 14)
    assert torch.equal(got, ref)              # the tile shape never changes results


def test_graph_refuses_to_launch_after_a_precision_change():
    """A precision change repacks (moves) the weights a graph points at: the
    graph refuses to launch instead of reading freed memory; a graph captured
    after the change replays the eager result, and a threshold change leaves
    an existing graph valid (it keeps its own threshold)."""
    spec, w = S.make_net("A", 1)
    net = dl.Net(S.serialize_weights(spec, w), precision="fp32")
    frames = S.render_frames(2, 96, 128, "tiny", 1004)
    buf = torch.from_numpy(frames).to(DEV)
    out = torch.zeros((2048, 8), dtype=torch.int32, device=DEV)
    counts = torch.zeros(3, dtype=torch.int32, device=DEV)
    g = net.graph(buf, out, counts)
    ref_out, ref_counts = eager(net, buf, 2048)
    net.set_config(precision="fp32", threshold=0.5)   # same precision: no repack
    g.launch()
    torch.cuda.synchronize()
    assert torch.equal(counts, ref_counts)            # the graph's own threshold (0.3)
    net.set_config(precision="bf16")
    with pytest.raises(dl.DlocError) as e:
        g.launch()
    assert e.value.code == dl.DL_ERR_INVALID_ARG
    g.close()
    g2 = net.graph(buf, out, counts)
    ref2_out, ref2_counts = eager(net, buf, 2048)
    counts.zero_()
    g2.launch()
    torch.cuda.synchronize()
    n = int(counts[-1].item())
    assert torch.equal(counts, ref2_counts) and torch.equal(out[:n], ref2_out)
    g2.close()
