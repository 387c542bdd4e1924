"""The allocation-free entry point (dl_localize_device_noalloc) through the C
ABI: the same records and counts as dl_localize_device on the same handle,
bit for bit, on two calls in a row (the second with a smaller batch, so the
fixed array keeps the first call's contents underneath), on a fresh handle
whose own workspace was never allocated, and in the BF16 form; batches past
its limits are refused before anything is queued."""
import numpy as np
import pytest

import smlm_synth as S

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no HIP device", allow_module_level=True)
import paper_2410_02314_amd as dl  # noqa: E402

DEV = torch.device("cuda:0")


def _run(net, frames, noalloc, cap=None):
    n, h, w = frames.shape
    fr = torch.from_numpy(np.ascontiguousarray(frames)).to(DEV)
    cap = cap or n * h * w // 8
    out = torch.full((cap, 8), -7, dtype=torch.int32, device=DEV)
    counts = torch.full((n + 1,), -1, dtype=torch.int32, device=DEV)
    torch.cuda.synchronize()
    (net.localize_device_noalloc if noalloc else net.localize_device)(fr, out, counts)
    torch.cuda.synchronize()
    c = counts.cpu().numpy().astype(np.int64)
    return dl.emitters_from_device(out, min(int(c[n]), cap)), c


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_noalloc_equals_localize_device_twice(prec):
    spec, w = S.make_net("A", 1)
    blob = S.serialize_weights(spec, w)
    big = S.render_frames(4, 128, 128, "tiny", 1001)
    small = S.render_frames(2, 72, 100, "tiny", 1002)
    ref = dl.Net(blob, precision=prec)
    want = [_run(ref, f, False) for f in (big, small)]
    print(f"noalloc {prec}: reference runs done", flush=True)
    net = dl.Net(blob, precision=prec)              # its own workspace is never allocated
    for f, (wr, wc) in zip((big, small), want):
        got, c = _run(net, f, True)
        assert np.array_equal(c, wc)
        assert np.array_equal(got, wr)
        assert len(got) > 20
    # the regular path still works on the same handle afterwards
    got, c = _run(net, big, False)
    assert np.array_equal(got, want[0][0])


def test_noalloc_refuses_batches_past_its_limits():
    spec, w = S.make_net("B", 2)
    net = dl.Net(S.serialize_weights(spec, w))
    fr = torch.zeros((1, 512, 512), dtype=torch.uint16, device=DEV)     # ~150 MiB of FP32 workspace
    out = torch.zeros((64, 8), dtype=torch.int32, device=DEV)
    counts = torch.zeros(2, dtype=torch.int32, device=DEV)
    with pytest.raises(dl.DlocError) as e:
        net.localize_device_noalloc(fr, out, counts)
    assert e.value.code == dl.DL_ERR_UNSUPPORTED and "workspace" in str(e.value)
    many = torch.zeros((dl.NOALLOC_MAX_FRAMES + 1, 8, 8), dtype=torch.uint16, device=DEV)
    c2 = torch.zeros(dl.NOALLOC_MAX_FRAMES + 2, dtype=torch.int32, device=DEV)
    with pytest.raises(dl.DlocError) as e:
        net.localize_device_noalloc(many, out, c2)
    assert e.value.code == dl.DL_ERR_UNSUPPORTED and "frames" in str(e.value)
    # the handle stays usable: a batch that fits runs
    small = torch.from_numpy(S.render_frames(1, 96, 96, "full", 5)).to(DEV)
    net.localize_device_noalloc(small, out, counts)
    torch.cuda.synchronize()
    assert int(counts[1].item()) >= 0
