"""The integer-valued networks that pin the reduced-precision forms bit for
bit (``tests/exact_nets.py``) have the properties those GPU tests rely on,
checked here with the oracle alone: every sum stays far below 2^24, the
emulated maps are integers, storing really rounds, FP8 weight scales are
exact powers of two that differ between output channels, and quantising the
weights leaves them unchanged."""
import numpy as np
import pytest

import oracle
from tests import exact_nets as X

DIL = (1, 2, 4, 8, 16)


@pytest.mark.parametrize("kind,C", [("bf16", 16), ("bf16", 48), ("fp8", 16), ("fp8", 48), ("fp8", 64)])
def test_exact_net_properties(kind, C):
    spec, w = X.fp8_exact_net(C, DIL, seed=21 + C) if kind == "fp8" else X.bf16_integer_net(C, DIL, seed=15 + C)
    frames = X.integer_frames(2, 70, 150, seed=7 + C)
    assert max(X.max_intermediate(f, spec, w) for f in frames) < 2 ** 22
    emu = np.stack([oracle.net_maps(f, spec, w, gain=1.0, offset=100.0, quant=kind) for f in frames])
    ex = np.stack([oracle.net_maps(f, spec, w, gain=1.0, offset=100.0) for f in frames])
    assert np.array_equal(emu, np.round(emu))
    assert np.mean(emu != ex) > 0.5                    # rounding of stored values propagates
    assert oracle.detect(emu[0, 0]).sum() > 10          # the detection stage is exercised
    if kind == "fp8":
        for k in range(len(DIL)):
            W = w[f"blk{k}.w1"].astype(np.float64)
            mx = np.abs(W).reshape(C, -1).max(1)
            live = mx > 0
            e = np.log2(mx[live] / 448.0)
            assert np.array_equal(e, np.round(e))        # exact power-of-two scales
            assert len(np.unique(e)) == 2                 # that differ between channels
            assert np.array_equal(oracle.quant_weights_fp8(W), W)
