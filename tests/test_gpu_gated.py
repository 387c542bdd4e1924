"""Gated localization: the tile gate decides per 256^2 tile, each conv layer
computes only what kept tiles need.  Checks:
* a gate that keeps every tile reproduces the ungated run bit for bit;
* a gate that keeps none gives no emitters;
* a mixed keep map: the GPU keep decisions equal the oracle gate's, maps on
  kept tiles equal the ungated maps bit for bit, and the emitter set equals the
  ungated set restricted to kept tiles except on kept-tile border pixels next
  to a skipped tile (there the skipped neighbours are absent from the local
  maximum test, which can only add detections).
"""
import math

import numpy as np
import pytest

import oracle
import smlm_synth as S

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no HIP device", allow_module_level=True)
import paper_2410_02314_amd as dl  # noqa: E402
from tests.test_gpu_fp32 import gpu_localize, gpu_maps  # noqa: E402

DEV = torch.device("cuda:0")


def brightness_gate(level, scale=50.0, thr=0.05):
    """g = scale * (max of ReLU(pooled x) - level) + logit(thr): keeps exactly
    the tiles whose brightest pooled pixel exceeds `level` at gate threshold
    `thr` (the gate's global pool is a max)."""
    th = np.zeros(673, np.float64)
    th[4] = 1.0                        # W1[0][0][1][1]: h1[0] = ReLU(p)
    th[80 + 4] = 1.0                   # W2[0][0][1][1]: h2[0] = ReLU(h1[0])
    th[664] = scale                    # fw[0]
    th[672] = -scale * level + math.log(thr / (1 - thr))   # fb
    return th


def oracle_pooled_tiles(frames):
    out = []
    for F in frames:
        x = oracle.preprocess(F, 0.5, 100.0, 0.01)
        for ty in range(F.shape[0] // 256):
            for tx in range(F.shape[1] // 256):
                p = oracle.gate_pool(x[ty * 256:(ty + 1) * 256, tx * 256:(tx + 1) * 256], 4)
                out.append(p)
    return np.stack(out)


def run(name, seed, frames, gate=None, thr=0.05):
    spec, w = S.make_net(name, seed)
    flags = dl.DL_FLAG_GATE if gate is not None else 0
    net = dl.Net(S.serialize_weights(spec, w), flags=flags)
    if gate is not None:
        net.set_gate(gate.astype(np.float32), thr)
    maps = gpu_maps(net, frames)
    rec, counts = gpu_localize(net, frames)
    keep = None
    if gate is not None:
        k = torch.zeros(len(frames) * (frames.shape[1] // 256) * (frames.shape[2] // 256), dtype=torch.uint8, device=DEV)
        net.gate_keep_map(k)
        torch.cuda.synchronize()
        keep = k.cpu().numpy().astype(bool)
    return spec, w, maps, rec, counts, keep


def test_keep_all_equals_ungated():
    frames = S.render_frames(2, 512, 768, "sparse", 4040)
    _, _, m0, r0, c0, _ = run("A", 1, frames)
    th = np.zeros(673)
    th[672] = 20.0
    _, _, m1, r1, c1, keep = run("A", 1, frames, th)
    assert keep.all()
    assert np.array_equal(m0, m1) and np.array_equal(r0, r1) and np.array_equal(c0, c1)


def test_keep_none_gives_nothing():
    frames = S.render_frames(1, 512, 512, "sparse", 4041)
    th = np.zeros(673)
    th[672] = -20.0
    _, _, _, rec, counts, keep = run("A", 1, frames, th)
    assert not keep.any() and len(rec) == 0 and counts[-1] == 0


@pytest.mark.parametrize("name", ["A", "B"])
def test_mixed_keep_map(name):
    frames = S.render_frames(2, 768, 1024, "sparse", 4042 if name == "A" else 4043)
    pooled = oracle_pooled_tiles(frames)
    peaks = np.maximum(pooled, 0).max(axis=(1, 2))
    srt = np.sort(peaks)
    gaps = np.diff(srt)
    mid = len(srt) // 4 + np.argmax(gaps[len(srt) // 4: 3 * len(srt) // 4])   # widest gap in the middle half
    level = 0.5 * (srt[mid] + srt[mid + 1])
    th = brightness_gate(level)
    ref_g = oracle.gate_forward(pooled, th)
    ref_keep = 1 / (1 + np.exp(-ref_g)) > 0.05
    spec, w, m0, r0, _, _ = run(name, 1 if name == "A" else 2, frames)
    _, _, m1, r1, _, keep = run(name, 1 if name == "A" else 2, frames, th)
    assert np.array_equal(keep, ref_keep)
    assert 0 < keep.sum() < keep.size
    gy, gx = frames.shape[1] // 256, frames.shape[2] // 256
    kmap = keep.reshape(len(frames), gy, gx)
    pix_keep = np.repeat(np.repeat(kmap, 256, axis=1), 256, axis=2)
    for f in range(len(frames)):
        kp = pix_keep[f]
        assert np.array_equal(m1[f][:, kp], m0[f][:, kp])          # kept tiles: exact ungated maps
    k0 = {(a, b, c) for a, b, c in zip(r0["frame"], r0["row"], r0["col"]) if pix_keep[a, b, c]}
    k1 = {(a, b, c) for a, b, c in zip(r1["frame"], r1["row"], r1["col"])}
    assert all(pix_keep[a, b, c] for a, b, c in k1)                 # nothing from skipped tiles
    assert k0 <= k1                                                 # gating never removes a kept detection
    for (a, b, c) in k1 - k0:                                        # extras sit next to a skipped tile
        nb = pix_keep[a, max(0, b - 1):b + 2, max(0, c - 1):c + 2]
        assert not nb.all()


def test_keep_map_belongs_to_the_most_recent_gated_run():
    """The keep flags live in the workspace the next run reuses: after an
    ungated run the keep map is refused rather than read stale."""
    frames = S.render_frames(1, 512, 512, "sparse", 4046)
    spec, w = S.make_net("A", 1)
    net = dl.Net(S.serialize_weights(spec, w), flags=dl.DL_FLAG_GATE)
    th = np.zeros(673, np.float32)
    th[672] = 20.0                                        # keeps every tile
    net.set_gate(th, 0.05)
    gpu_localize(net, frames)
    k = torch.zeros(4, dtype=torch.uint8, device=DEV)
    assert net.gate_keep_map(k) == 4                     # four 256^2 tiles
    torch.cuda.synchronize()
    assert k.cpu().numpy().all()
    net.set_gate(None)                                    # the next run is ungated
    gpu_localize(net, frames)
    with pytest.raises(dl.DlocError) as e:
        net.gate_keep_map(k)
    assert e.value.code == dl.DL_ERR_INVALID_ARG
