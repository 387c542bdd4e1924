"""Reduced-precision forms (BF16 and FP8 block convolutions, FP32
accumulation) on realistic networks: accuracy reports.

Their parity is pinned bit for bit in ``test_gpu_exact.py`` (integer-valued
networks on which every sum is exact, so the only rounding is the form's
own).  On real weights the FP32 and FP64 accumulations of the GPU and the
emulation land on opposite sides of some rounding boundaries and the
differences propagate, so these tests report how close the GPU stays to the
oracle's emulation and to the exact FP64 oracle, and guard that level:

* maps: the GPU's error against the emulation is no more than twice the
  emulation's own error against the exact oracle;
* emitters (matched one-to-one within 1 px): recall, precision and RMS offset
  differences against the exact oracle, held to the level of the oracle's own
  emulation of the form.
"""
import numpy as np
import pytest

import oracle
import smlm_synth as S
from tests.parity import map_rel_err, match_by_distance

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no HIP device", allow_module_level=True)
import paper_2410_02314_amd as dl  # noqa: E402
from tests.test_gpu_fp32 import gpu_localize, gpu_maps  # noqa: E402


def integer_net(C=16, dil=(1, 2), seed=15):
    spec = S.NetSpec("int", C, dil, in_scale=1.0)
    r = np.random.default_rng(seed)
    w = {}
    for n, s in S.tensor_layout(spec):
        if n.endswith(("w1", "w2")):
            w[n] = (r.integers(-1, 3, size=s) * (r.random(s) < 0.08)).astype(np.float32)
        elif n == "stem.w":
            w[n] = r.integers(0, 2, size=s).astype(np.float32)
        else:
            w[n] = r.integers(-1, 2, size=s).astype(np.float32)
    return spec, w


def test_bf16_integer_net_bit_exact_vs_emulation():
    spec, w = integer_net()
    r = np.random.default_rng(3)
    frames = (100 + r.integers(0, 20, size=(2, 37, 70))).astype(np.uint16)
    net = dl.Net(S.serialize_weights(spec, w), precision="bf16", gain=1.0, offset=100.0)
    got = gpu_maps(net, frames)
    emu = np.stack([oracle.net_maps(f, spec, w, gain=1.0, offset=100.0, quant="bf16") for f in frames])
    ex = np.stack([oracle.net_maps(f, spec, w, gain=1.0, offset=100.0) for f in frames])
    assert np.abs(ex).max() < 2 ** 24                 # every sum exact in FP32 too
    assert not np.array_equal(emu, ex)                # rounding of stored values really happens
    assert np.array_equal(got, emu)


def _setup(prec, name="A", seed=1, frames_seed=1001, n=4, h=128, w=128, model="tiny"):
    spec, wts = S.make_net(name, seed)
    net = dl.Net(S.serialize_weights(spec, wts), precision=prec)
    frames = S.render_frames(n, h, w, model, frames_seed)
    return spec, wts, net, frames


def test_bf16_close_to_emulation():
    spec, wts, net, frames = _setup("bf16")
    got = gpu_maps(net, frames)
    emu = oracle.net_maps_batch(frames, spec, wts, quant="bf16")
    ex = oracle.net_maps_batch(frames, spec, wts)
    e_gpu = map_rel_err(got, emu)
    e_emu = map_rel_err(emu, ex)
    print("gpu vs emulation", e_gpu, "emulation vs exact", e_emu)
    assert np.all(e_gpu <= 2.0 * e_emu + 1e-4)


@pytest.mark.parametrize("name,model,n,side", [("A", "tiny", 4, 128), ("B", "full", 2, 256)])
def test_bf16_accuracy_vs_fp64(name, model, n, side):
    spec, wts, net, frames = _setup("bf16", name, 1 if name == "A" else 2, 1001, n, side, side, model)
    ref = oracle.localize(frames, spec, wts)
    emu = oracle.localize(frames, spec, wts, quant="bf16")
    rec, counts = gpu_localize(net, frames)
    got = match_by_distance(rec, ref, 1.0)
    base = match_by_distance(emu, ref, 1.0)
    print({"gpu_bf16": got, "oracle_bf16_emulation": base})
    assert got["recall"] >= min(0.99, base["recall"] - 0.01)
    assert got["precision"] >= min(0.99, base["precision"] - 0.01)
    assert got["rms_dx_px"] <= max(0.15, 1.5 * base["rms_dx_px"])
    assert got["rms_dy_px"] <= max(0.15, 1.5 * base["rms_dy_px"])


def test_bf16_full_size_tiling_invariance_and_window():
    """Net B, BF16, a 2048 x 2048 frame; tile shape does not change the result."""
    spec, wts, net, frames = _setup("bf16", "B", 2, 1002, n=1, h=2048, w=2048, model="full")
    got = gpu_maps(net, frames)
    net4 = dl.Net(S.serialize_weights(spec, wts), precision="bf16", tile_rows=4)
    assert np.array_equal(got, gpu_maps(net4, frames))
    y0, x0, hh, ww = 900, 1100, 32, 48
    emu = oracle.net_maps_window(frames[0], spec, wts, y0, x0, hh, ww, quant="bf16")
    ex = oracle.net_maps_window(frames[0], spec, wts, y0, x0, hh, ww)
    assert np.all(map_rel_err(got[0, :, y0:y0 + hh, x0:x0 + ww], emu) <= 2.0 * map_rel_err(emu, ex) + 1e-4)


# ------------------------------------------------------------------ FP8
@pytest.mark.parametrize("name,model,n,side", [("A", "tiny", 4, 128), ("B", "full", 2, 256)])
def test_fp8_close_to_emulation_and_accuracy(name, model, n, side):
    """FP8 e4m3 block convolutions (per-output-channel weight scales, stored
    activations with one power-of-two scale per 32-channel group of each
    pixel, FP32 accumulation) against the oracle's FP8 emulation and the exact
    FP64 oracle."""
    spec, wts, net, frames = _setup("fp8", name, 1 if name == "A" else 2, 1001, n, side, side, model)
    got = gpu_maps(net, frames)
    emu = oracle.net_maps_batch(frames, spec, wts, quant="fp8")
    ex = oracle.net_maps_batch(frames, spec, wts)
    e_gpu, e_emu = map_rel_err(got, emu), map_rel_err(emu, ex)
    print("fp8: gpu vs emulation", e_gpu, "emulation vs exact", e_emu)
    assert np.all(e_gpu <= 2.0 * e_emu + 1e-4)
    ref = oracle.localize(frames, spec, wts)
    emu_rec = oracle.localize(frames, spec, wts, quant="fp8")
    rec, _ = gpu_localize(net, frames)
    g = match_by_distance(rec, ref, 1.0)
    b = match_by_distance(emu_rec, ref, 1.0)
    print({"gpu_fp8": g, "oracle_fp8_emulation": b})
    assert g["recall"] >= b["recall"] - 0.02 and g["precision"] >= b["precision"] - 0.02


def test_fp8_tiling_invariance():
    """Activation scales are per pixel and channel group, so the tile shape does
    not change FP8 results."""
    spec, wts, net, frames = _setup("fp8", "B", 2, 1002, n=2, h=320, w=448, model="full")
    net4 = dl.Net(S.serialize_weights(spec, wts), precision="fp8", tile_rows=4)
    assert np.array_equal(gpu_maps(net, frames), gpu_maps(net4, frames))
