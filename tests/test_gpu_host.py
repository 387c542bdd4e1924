"""Host-memory entry points: dl_localize (copy in, localize, copy out) and the
pipelined form (batch k+1 copied on a side stream while batch k is processed)
give exactly the device-resident results, with pageable or pinned frames and
with the overlap on or off; capacity overflow follows the two-call protocol."""
import ctypes

import numpy as np
import pytest

import smlm_synth as S

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no HIP device", allow_module_level=True)
import paper_2410_02314_amd as dl  # noqa: E402
from tests.test_gpu_fp32 import gpu_localize  # noqa: E402


def test_host_localize_equals_device_path():
    spec, w = S.make_net("A", 1)
    net = dl.Net(S.serialize_weights(spec, w))
    frames = S.render_frames(3, 200, 256, "tiny", 61)
    dev_rec, _ = gpu_localize(net, frames)
    host_rec = net.localize(frames)
    assert np.array_equal(host_rec, dev_rec)


@pytest.mark.parametrize("pinned", [False, True])
def test_pipelined_batches_overlap_on_off(pinned):
    spec, w = S.make_net("B", 2)
    net = dl.Net(S.serialize_weights(spec, w), precision="bf16")
    frames = S.render_frames(12, 256, 256, "full", 62).reshape(3, 4, 256, 256)
    ref = []
    for k in range(3):
        r, _ = gpu_localize(net, frames[k])
        r = r.copy()
        r["frame"] += 4 * k
        ref.append(r)
    ref = np.concatenate(ref)
    src, pin = frames, None
    if pinned:
        pin = dl.host_alloc(frames.nbytes)
        buf = (ctypes.c_char * frames.nbytes).from_address(pin)
        src = np.frombuffer(buf, dtype=np.uint16).reshape(frames.shape)
        src[...] = frames
    try:
        for overlap in (True, False):
            got = net.localize_pipelined(src, overlap=overlap)
            assert np.array_equal(got, ref), overlap
    finally:
        if pin:
            dl.host_free(pin)


def test_host_capacity_protocol():
    spec, w = S.make_net("A", 1)
    net = dl.Net(S.serialize_weights(spec, w))
    frames = S.render_frames(2, 128, 128, "tiny", 63)
    full = net.localize(frames)
    out = np.empty(5, dl.EMITTER_DTYPE)
    cnt = ctypes.c_size_t()
    F = np.ascontiguousarray(frames)
    rc = dl.lib().dl_localize(net.handle, F.ctypes.data, 2, 128, 128, out.ctypes.data, 5, ctypes.byref(cnt))
    assert rc == dl.DL_ERR_CAPACITY and cnt.value == len(full)
    assert np.array_equal(out, full[:5])


@pytest.mark.parametrize("overlap", [1, 0])
def test_pipelined_capacity_inside_a_later_batch(overlap):
    """The capacity runs out inside batch 2 while batch 1 is still being
    collected (overlap on): the first `cap` records and the total count are
    those of the uncapped call."""
    spec, w = S.make_net("A", 1)
    net = dl.Net(S.serialize_weights(spec, w))
    frames = S.render_frames(6, 128, 192, "tiny", 64).reshape(3, 2, 128, 192)
    full = net.localize_pipelined(frames, overlap=bool(overlap))
    per = [len(net.localize(frames[k])) for k in range(3)]
    assert sum(per) == len(full) and per[0] > 0 and per[2] > 1
    cap = per[0] + per[1] + per[2] // 2
    out = np.empty(cap, dl.EMITTER_DTYPE)
    cnt = ctypes.c_size_t()
    F = np.ascontiguousarray(frames)
    rc = dl.lib().dl_localize_pipelined(net.handle, F.ctypes.data, 3, 2, 128, 192, overlap, out.ctypes.data,
                                        cap, ctypes.byref(cnt))
    assert rc == dl.DL_ERR_CAPACITY and cnt.value == len(full)
    assert np.array_equal(out, full[:cap])


def test_pipelined_slots_grow_then_serve_smaller_batches():
    """The handle's frame and record slots grow for a larger call and are
    reused by a smaller one; each call equals its own device-path result."""
    spec, w = S.make_net("A", 1)
    net = dl.Net(S.serialize_weights(spec, w))
    for n, h, wd, seed in ((1, 96, 128, 65), (3, 256, 320, 66), (2, 64, 80, 67)):
        frames = S.render_frames(2 * n, h, wd, "tiny", seed).reshape(2, n, h, wd)
        ref = []
        for k in range(2):
            r, _ = gpu_localize(net, frames[k])
            r = r.copy()
            r["frame"] += n * k
            ref.append(r)
        got = net.localize_pipelined(frames, overlap=True)
        assert np.array_equal(got, np.concatenate(ref)), (n, h, wd)
