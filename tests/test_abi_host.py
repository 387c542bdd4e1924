"""C-ABI host tests: no GPU needed.  The library loads, exports every function
declared in include/dloc.h, parses weights blobs, and rejects bad arguments
before any HIP call."""
import ctypes
import math
import os
import re
import struct

import numpy as np
import pytest

import smlm_synth as S

dl = pytest.importorskip("paper_2410_02314_amd")
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "dloc.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(dl_[a-z0-9_]+)\s*\(", txt)))


def test_every_declared_symbol_is_exported():
    names = header_functions()
    assert len(names) >= 15
    L = ctypes.CDLL(dl.LIB_PATH)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_abi_version_and_defaults():
    assert dl.abi_version() == 3
    c = dl.DLConfig()
    assert dl.lib().dl_default_config(ctypes.byref(c)) == 0
    assert (c.precision, c.device, c.flags, c.tile_rows) == (0, 0, 0, 0)
    assert abs(c.threshold - 0.3) < 1e-7 and c.gain == 0.5 and c.offset == 100.0
    assert dl.lib().dl_default_config(None) == dl.DL_ERR_INVALID_ARG


def blob(name="A", seed=1):
    spec, w = S.make_net(name, seed)
    return spec, w, S.serialize_weights(spec, w)


@pytest.mark.parametrize("name", ["A", "B", "AU", "BU"])
def test_inspect_weights_reads_header(name):
    spec, w, b = blob(name, 1 if name[0] == "A" else 2)
    info = dl.inspect_weights(b)
    assert info["C"] == spec.C and info["dilations"] == spec.dilations
    assert info["nparams"] == S.param_count(spec)
    assert info["head_outputs"] == spec.head_outputs
    assert info["receptive_radius"] == S.receptive_radius(spec)
    assert math.isclose(info["in_scale"], spec.in_scale, rel_tol=1e-7)
    assert info["z_scale"] == spec.z_scale and info["ph_scale"] == spec.ph_scale


def _code(b):
    info = dl.DLNetInfo()
    buf = ctypes.create_string_buffer(bytes(b), len(b))
    return dl.lib().dl_inspect_weights(buf, len(b), ctypes.byref(info))


def test_bad_blobs_are_rejected():
    spec, w, b = blob("A")
    assert _code(b) == 0
    assert _code(b"XXXX" + b[4:]) == dl.DL_ERR_BAD_WEIGHTS              # magic
    assert _code(b[:-4]) == dl.DL_ERR_BAD_WEIGHTS                        # truncated
    assert _code(b + b"\0\0\0\0") == dl.DL_ERR_BAD_WEIGHTS               # trailing bytes
    assert _code(b[:40]) == dl.DL_ERR_BAD_WEIGHTS                        # shorter than header
    bad = bytearray(b); bad[4:8] = struct.pack("<I", 2)
    assert _code(bad) == dl.DL_ERR_BAD_WEIGHTS                           # version
    bad = bytearray(b); bad[8:12] = struct.pack("<I", 24)
    assert _code(bad) == dl.DL_ERR_UNSUPPORTED                           # C
    bad = bytearray(b); bad[12:16] = struct.pack("<I", 0)
    assert _code(bad) == dl.DL_ERR_BAD_WEIGHTS                           # nblocks
    bad = bytearray(b); bad[16:20] = struct.pack("<I", 0)
    assert _code(bad) == dl.DL_ERR_BAD_WEIGHTS                           # dilation 0
    bad = bytearray(b); bad[48:52] = struct.pack("<f", -1.0)
    assert _code(bad) == dl.DL_ERR_BAD_WEIGHTS                           # in_scale
    bad = bytearray(b); bad[100:104] = struct.pack("<f", float("nan"))
    assert _code(bad) == dl.DL_ERR_BAD_WEIGHTS                           # NaN weight
    assert "NaN" in dl.last_error()
    bad = bytearray(b); bad[60:64] = struct.pack("<I", 7)
    assert _code(bad) == dl.DL_ERR_BAD_WEIGHTS                           # head outputs not 5 or 10
    bad = bytearray(b); bad[60:64] = struct.pack("<I", 10)
    assert _code(bad) == dl.DL_ERR_BAD_WEIGHTS                           # 10 outputs: blob too short
    bad = bytearray(b); bad[60:64] = struct.pack("<I", 5)
    assert _code(bad) == 0                                               # 5 written out
    assert dl.lib().dl_inspect_weights(None, 10, ctypes.byref(dl.DLNetInfo())) == dl.DL_ERR_INVALID_ARG


def test_inspect_dense_blob_reads_header():
    spec, w, b = blob("D", 3)
    assert b[:4] == b"DLD1" and len(b) == 80 + 4 * S.param_count(spec)
    info = dl.inspect_weights(b)
    assert info["C"] == 32 and info["dilations"] == (2, 4, 8, 16) and info["head_outputs"] == 5
    assert info["dense_layers"] == 4 and info["dense_growth"] == 16
    assert info["nparams"] == S.param_count(spec) == 142181
    assert info["receptive_radius"] == S.receptive_radius(spec) == 121
    assert math.isclose(info["in_scale"], spec.in_scale, rel_tol=1e-7)
    r = blob("A")[2]
    assert dl.inspect_weights(r)["dense_layers"] == 0 and dl.inspect_weights(r)["dense_growth"] == 0


def test_bad_dense_blobs_are_rejected():
    """DLD1 header: magic, version @4, C @8, nblocks @12, layers @16, growth @20,
    dilation[8] @24, in_scale @56, z_scale @60, ph_scale @64, head outputs @68."""
    spec, w, b = blob("D", 3)
    assert _code(b) == 0
    assert _code(b[:-4]) == dl.DL_ERR_BAD_WEIGHTS
    assert _code(b + b"\0" * 4) == dl.DL_ERR_BAD_WEIGHTS
    assert _code(b[:70]) == dl.DL_ERR_BAD_WEIGHTS
    for off, val, code in [(4, 2, dl.DL_ERR_BAD_WEIGHTS),            # version
                           (8, 48, dl.DL_ERR_UNSUPPORTED),           # C
                           (12, 0, dl.DL_ERR_BAD_WEIGHTS),           # no blocks
                           (12, 9, dl.DL_ERR_BAD_WEIGHTS),           # more blocks than descriptors hold
                           (16, 0, dl.DL_ERR_BAD_WEIGHTS),           # no layers
                           (16, 9, dl.DL_ERR_BAD_WEIGHTS),
                           (20, 24, dl.DL_ERR_UNSUPPORTED),          # growth
                           (24, 0, dl.DL_ERR_BAD_WEIGHTS),           # dilation 0
                           (68, 7, dl.DL_ERR_BAD_WEIGHTS),           # head outputs
                           (16, 3, dl.DL_ERR_BAD_WEIGHTS)]:          # other layer count: wrong length
        bad = bytearray(b)
        bad[off:off + 4] = struct.pack("<I", val)
        assert _code(bad) == code, (off, val)
    bad = bytearray(b); bad[56:60] = struct.pack("<f", 0.0)
    assert _code(bad) == dl.DL_ERR_BAD_WEIGHTS
    bad = bytearray(b); bad[200:204] = struct.pack("<f", float("inf"))
    assert _code(bad) == dl.DL_ERR_BAD_WEIGHTS


def _create(b, **cfg):
    c = dl.make_config(**cfg)
    h = ctypes.c_void_p()
    buf = ctypes.create_string_buffer(bytes(b), len(b))
    rc = dl.lib().dl_create_net(buf, len(b), ctypes.byref(c), ctypes.byref(h))
    if rc == 0:
        dl.lib().dl_destroy_net(h)
    return rc


@pytest.mark.parametrize("cfg", [dict(precision=7), dict(threshold=0.0), dict(threshold=1.0),
                                 dict(gain=0.0), dict(gain=float("nan")), dict(offset=float("inf")),
                                 dict(device=-1), dict(tile_rows=5), dict(flags=0x80),
                                 dict(in_scale_override=-0.01), dict(in_scale_override=float("inf")),
                                 dict(tile_w=-1), dict(tile_queue=3), dict(tile_queue=-1)])
def test_create_rejects_bad_config_before_device(cfg):
    _, _, b = blob("A")
    assert _create(b, **cfg) == dl.DL_ERR_INVALID_ARG


@pytest.mark.parametrize("prec,tw", [("fp32", 64), ("bf16", 32), ("fp8", 48)])
def test_create_refuses_tile_widths_not_built(prec, tw):
    _, _, b = blob("A")
    assert _create(b, precision=prec, tile_w=tw) == dl.DL_ERR_UNSUPPORTED


@pytest.mark.parametrize("cfg", [dict(precision="bf16"), dict(precision="fp8"), dict(precision="bf16x3"),
                                 dict(tile_rows=8), dict(tile_w=32), dict(flags=1)])
def test_create_refuses_what_the_dense_kernels_do_not_run(cfg):
    """FP32 only, their fixed tile, no tile gate: refused before any device call."""
    _, _, b = blob("D", 3)
    assert _create(b, **cfg) == dl.DL_ERR_UNSUPPORTED
    if "tile_w" not in cfg:             # (a width no form is built for is refused earlier)
        assert "dense" in dl.last_error()


@pytest.mark.parametrize("q", [1, 2])
def test_tile_queue_is_refused_for_the_residual_kernels(q):
    _, _, b = blob("A")
    assert _create(b, tile_queue=q) == dl.DL_ERR_UNSUPPORTED
    assert "tile_queue" in dl.last_error()


def test_create_rejects_bad_blob_and_null_pointers():
    _, _, b = blob("A")
    assert _create(b[:-1]) == dl.DL_ERR_BAD_WEIGHTS
    h = ctypes.c_void_p()
    assert dl.lib().dl_create_net(None, 100, None, ctypes.byref(h)) == dl.DL_ERR_INVALID_ARG
    buf = ctypes.create_string_buffer(bytes(b), len(b))
    assert dl.lib().dl_create_net(buf, len(b), None, None) == dl.DL_ERR_INVALID_ARG


def test_calls_on_null_handle_fail_cleanly():
    L = dl.lib()
    assert L.dl_localize_device(None, 16, 1, 8, 8, None, 16, 4, 16) == dl.DL_ERR_INVALID_ARG
    assert L.dl_maps_device(None, 16, 1, 8, 8, None, 16) == dl.DL_ERR_INVALID_ARG
    assert L.dl_localize_device_noalloc(None, 16, 1, 8, 8, None, 16, 4, 16) == dl.DL_ERR_INVALID_ARG
    assert L.dl_debug_compact(None, 16, 16, 1, 8, 8, None, 16, 4, 16) == dl.DL_ERR_INVALID_ARG
    assert L.dl_localize_maps(None, 16, 1, 8, 8, 16) == dl.DL_ERR_INVALID_ARG
    assert L.dl_localize_rois(None, None, 1, None, 0, None) == dl.DL_ERR_INVALID_ARG
    assert L.dl_set_config(None, None) == dl.DL_ERR_INVALID_ARG
    assert L.dl_profile_enable(None, 1) == dl.DL_ERR_INVALID_ARG
    assert L.dl_host_alloc(0, ctypes.byref(ctypes.c_void_p())) == dl.DL_ERR_INVALID_ARG
    assert "bytes is 0" in dl.last_error()
    L.dl_destroy_net(None)                       # no-op
    L.dl_host_free(None)                         # no-op


def test_create_without_gpu_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    _, _, b = blob("B")
    assert _create(b) == dl.DL_ERR_DEVICE


def test_measure_rate_rejects_bad_requests_before_any_hip_call():
    v = ctypes.c_double()
    L = dl.lib()
    assert L.dl_measure_rate(7, 0, 1, ctypes.byref(v)) == dl.DL_ERR_INVALID_ARG      # unknown kind
    assert L.dl_measure_rate(-1, 0, 1, ctypes.byref(v)) == dl.DL_ERR_INVALID_ARG
    assert L.dl_measure_rate(3, 100, 1, ctypes.byref(v)) == dl.DL_ERR_INVALID_ARG    # copy size not 16-aligned
    assert L.dl_measure_rate(3, 0, 1, ctypes.byref(v)) == dl.DL_ERR_INVALID_ARG
    assert L.dl_measure_rate(0, 0, 0, ctypes.byref(v)) == dl.DL_ERR_INVALID_ARG      # no repetition
    assert L.dl_measure_rate(0, 0, 1, None) == dl.DL_ERR_INVALID_ARG


def test_set_camera_maps_rejects_a_null_handle():
    g = np.full((4, 4), 0.5, np.float32)
    assert dl.lib().dl_set_camera_maps(None, g.ctypes.data, g.ctypes.data, 4, 4) == dl.DL_ERR_INVALID_ARG
