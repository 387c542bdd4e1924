"""Reduced-precision forms held to the oracle's emulation bit for bit.

On the integer-valued networks of ``tests/exact_nets.py`` every product and
sum is exact in FP32 and FP64, so the only rounding is where a form stores a
value (BF16: 8 significant bits; FP8 e4m3: 4, with a power-of-two scale per
32-channel group of each pixel) and where FP8 scales weights (exact powers of
two here, different per output channel).  The GPU's maps must then equal the
oracle's BF16 / FP8 emulation exactly, for every channel count the kernels
support, every dilation of the benchmark network (1, 2, 4, 8, 16: the plain
and all phase layouts), ragged frames spanning several tiles, uniform batches
and uneven ROI lists.  Detections follow from the maps, so the emitter sets
must be identical too.
"""
import numpy as np
import pytest

import oracle
from tests import exact_nets as X

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no HIP device", allow_module_level=True)
import paper_2410_02314_amd as dl  # noqa: E402
from tests.test_gpu_fp32 import gpu_localize, gpu_maps  # noqa: E402

DEV = torch.device("cuda:0")
DIL = (1, 2, 4, 8, 16)


def _net(kind, C):
    if kind == "fp8":
        return X.fp8_exact_net(C, DIL, seed=21 + C)
    # split BF16 on integers: hi and lo are integers and every product of the
    # three terms is exact, so only the split's own rounding (the dropped lo
    # bits of values above 2^16 and the lo xl term) separates it from exact
    return X.bf16_integer_net(C, DIL, seed=15 + C)


def _make(spec, w, prec, **cfg):
    import smlm_synth as S
    return dl.Net(S.serialize_weights(spec, w), precision=prec, gain=1.0, offset=100.0, **cfg)


# every channel count each form's kernel is built for (BF16 with C = 64 does
# not fit its tile and weights in LDS; dl_create_net refuses it)
CASES = [("bf16", 16), ("bf16", 32), ("bf16", 48), ("fp8", 16), ("fp8", 32), ("fp8", 48), ("fp8", 64),
         ("bf16x3", 16), ("bf16x3", 32), ("bf16x3", 48)]


@pytest.mark.parametrize("kind,C", CASES)
def test_integer_net_bit_exact_vs_emulation(kind, C):
    spec, w = _net(kind, C)
    frames = X.integer_frames(2, 70, 150, seed=7 + C)
    assert max(X.max_intermediate(f, spec, w) for f in frames) < 2 ** 22
    net = _make(spec, w, kind)
    print(f"{kind} C={C}: case built, running", flush=True)
    got = gpu_maps(net, frames)
    emu = np.stack([oracle.net_maps(f, spec, w, gain=1.0, offset=100.0, quant=kind) for f in frames])
    ex = np.stack([oracle.net_maps(f, spec, w, gain=1.0, offset=100.0) for f in frames])
    assert not np.array_equal(emu, ex)               # the form's rounding really happens
    bad = np.argwhere(got != emu)
    assert bad.size == 0, (len(bad), bad[:5], got[tuple(bad[0])], emu[tuple(bad[0])])
    # detections: the same set as the oracle's on the same maps
    rec, counts = gpu_localize(net, frames)
    for f in range(frames.shape[0]):
        det = oracle.detect(emu[f, 0].astype(np.float64))
        g = rec[rec["frame"] == f]
        gd = np.zeros_like(det)
        gd[g["row"], g["col"]] = True
        assert np.array_equal(gd, det), f
        assert counts[f] == det.sum()


def test_bf16_c64_is_refused():
    spec, w = X.bf16_integer_net(64, DIL)
    import smlm_synth as S
    with pytest.raises(dl.DlocError) as e:
        dl.Net(S.serialize_weights(spec, w), precision="bf16")
    assert e.value.code == dl.DL_ERR_UNSUPPORTED


@pytest.mark.parametrize("kind", ["bf16", "fp8", "bf16x3"])
def test_integer_net_tile_shapes_agree(kind):
    """4-row and 8-row conv tiles give the same bits (and both equal the
    emulation, by the test above)."""
    spec, w = _net(kind, 48)
    frames = X.integer_frames(2, 45, 131, seed=99)
    a = gpu_maps(_make(spec, w, kind, tile_rows=8), frames)
    b = gpu_maps(_make(spec, w, kind, tile_rows=4), frames)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("kind", ["bf16", "fp8", "bf16x3"])
def test_integer_net_uneven_rois_bit_exact(kind):
    """Uneven ROI lists (one launch per layer over all ROIs, some strided out
    of a larger frame) equal the emulation ROI by ROI."""
    spec, w = X.fp8_exact_net(32, (1, 2, 4), seed=5) if kind == "fp8" else X.bf16_integer_net(32, (1, 2, 4), seed=6)
    shapes = [(64, 96), (128, 64), (33, 200), (1, 130), (200, 37), (17, 5), (90, 90)]
    rois = [X.integer_frames(1, h, wd, seed=300 + k)[0] for k, (h, wd) in enumerate(shapes)]
    big = X.integer_frames(1, 150, 260, seed=77)[0]
    big_t = torch.from_numpy(big).to(DEV)
    cut = [(10, 20, 64, 100), (80, 150, 70, 110)]          # (y0, x0, h, w) views with row stride 260
    dev = [torch.from_numpy(np.ascontiguousarray(r)).to(DEV) for r in rois]
    dev += [big_t[y0:y0 + hh, x0:x0 + ww] for y0, x0, hh, ww in cut]
    rois += [big[y0:y0 + hh, x0:x0 + ww] for y0, x0, hh, ww in cut]
    net = _make(spec, w, kind)
    total = sum(r.shape[0] * r.shape[1] for r in rois)
    maps = torch.full((5 * total,), float("nan"), dtype=torch.float32, device=DEV)
    net.maps_rois_device(dev, maps)
    torch.cuda.synchronize()
    m = maps.cpu().numpy()
    o = 0
    for k, r in enumerate(rois):
        hh, ww = r.shape
        got = m[o:o + 5 * hh * ww].reshape(5, hh, ww)
        o += 5 * hh * ww
        emu = oracle.net_maps(np.ascontiguousarray(r), spec, w, gain=1.0, offset=100.0, quant=kind)
        assert np.array_equal(got, emu), (k, r.shape, int((got != emu).sum()))
