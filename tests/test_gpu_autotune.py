"""The autotuner with its cache (dl_autotune_ex): it times strip widths of the
tile order and each block's tile rows on the caller's batch, applies the
fastest, and records it as a JSON line keyed by device, net, precision and
batch shape; a second call with the cache applies the line without timing.
Every tiling it can choose gives the same bits (the per-pixel arithmetic does
not depend on the tile), checked here for hand-written cache lines with each
strip width and mixed per-block rows, against the default tiling and the
oracle."""
import json

import numpy as np
import pytest

import oracle
import smlm_synth as S
from tests.parity import map_rel_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no HIP device", allow_module_level=True)
import paper_2410_02314_amd as dl  # noqa: E402
from tests.test_gpu_fp32 import gpu_localize, gpu_maps  # noqa: E402

DEV = torch.device("cuda:0")


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_tuner_cache_roundtrip_and_every_tiling_gives_the_same_bits(prec, tmp_path):
    spec, w = S.make_net("B", 2)
    blob = S.serialize_weights(spec, w)
    frames = S.render_frames(2, 320, 384, "full", 96)
    d = torch.from_numpy(frames).to(DEV)
    base = dl.Net(blob, precision=prec)
    want_maps = gpu_maps(base, frames)
    want_rec, _ = gpu_localize(base, frames)
    cache = tmp_path / "tune.jsonl"
    net = dl.Net(blob, precision=prec)
    r1 = net.autotune_ex(d, reps=2, cache_path=str(cache))
    print(r1, flush=True)
    assert not r1["from_cache"] and r1["configs_timed"] == 4 + len(spec.dilations)
    assert all(r in (4, 8) for r in r1["rows"]) and r1["strip"] in (4, 8, 16, 32)
    assert 0 < r1["ms_best"] <= r1["ms_default"] * 1.01
    lines = [json.loads(l) for l in cache.read_text().splitlines()]
    assert len(lines) == 1 and lines[0]["rows"] == r1["rows"] and lines[0]["strip"] == r1["strip"]
    assert "batch=2x320x384" in lines[0]["key"] and f"prec={dl.PRECISIONS[prec]}" in lines[0]["key"]
    assert np.array_equal(gpu_maps(net, frames), want_maps)
    # a second handle takes the cached tiling without timing anything
    net2 = dl.Net(blob, precision=prec)
    r2 = net2.autotune_ex(d, reps=2, cache_path=str(cache))
    assert r2["from_cache"] and r2["configs_timed"] == 0 and r2["rows"] == r1["rows"] and r2["strip"] == r1["strip"]
    # hand-written cache lines: every strip width, mixed per-block rows, after a
    # line the parser must skip
    key = lines[0]["key"]
    for strip, rows in ((4, [4, 8, 4, 8, 4]), (16, [8, 4, 8, 4, 8]), (32, [4, 4, 4, 4, 8]), (8, [8] * 5)):
        c2 = tmp_path / f"hand{strip}.jsonl"
        c2.write_text('{"key": "other", "rows": [8], "strip": 8, "ms": 1}\n'
                      + json.dumps({"key": key, "rows": rows, "strip": strip, "ms": 1.0}) + "\n")
        n3 = dl.Net(blob, precision=prec)
        r3 = n3.autotune_ex(d, reps=1, cache_path=str(c2))
        assert r3["from_cache"] and r3["rows"] == rows and r3["strip"] == strip
        assert np.array_equal(gpu_maps(n3, frames), want_maps), (strip, rows)
        rec, _ = gpu_localize(n3, frames)
        assert np.array_equal(rec, want_rec), (strip, rows)
    if prec == "fp32":
        ref = oracle.net_maps_batch(frames, spec, w)
        assert map_rel_err(want_maps, ref).max() <= 1e-4
