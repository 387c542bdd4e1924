"""The oracle's pins catch plausible mistakes.  Each case plants one mistake
in a copy of oracle.c: a transposed kernel, a dropped dilation, a dropped bias
or residual, a wrong sign, a reversed tie-break, truncating BF16 rounding, an
FP8 group scale one power of two off, an FP8 weight scale taken over the
whole tensor or applied the wrong way, an FP8 rounding point dropped or
added, the gate's gradient sent to the last maximum, swapped camera maps, a
dropped head bias, the dense blocks' and the U-Net's wiring.  It builds the copy with the
oracle's own flags, points the oracle module at it, and checks that at least
one of the named pins fails.  The planted copy lives in a temporary directory;
the real oracle is restored afterwards.

The post-processing written in Python (records, softplus, uncertainties, the
sigma filter, the threshold's logit) gets the same treatment: a mistake is
planted in one function's source, the changed function replaces the oracle's
for the duration of the test, and a named pin must fail."""
import inspect
import subprocess
import textwrap

import numpy as np

import pytest

import oracle
import smlm_synth as S
from tests import test_oracle_bf16x3 as B3
from tests import test_oracle_camera as CAM
from tests import test_oracle_dense as DN
from tests import test_oracle_fp8 as FP8
from tests import test_oracle_pins as PINS
from tests import test_oracle_train as TR
from tests import test_oracle_uncertainty as UNC
import oracle.train  # noqa: E402,F401

MUTANTS = [
    ("transposed 3x3 kernel",
     "double wt = W[(((long)o * cin + c) * 3 + (u + 1)) * 3 + (v + 1)];",
     "double wt = W[(((long)o * cin + c) * 3 + (v + 1)) * 3 + (u + 1)];",
     [(PINS.test_conv_delta_input_reproduces_weights, (2,))]),
    ("row dilation dropped",
     "int ii = i + d * u;",
     "int ii = i + u;",
     [(PINS.test_conv_matches_torch_float64, (4,))]),
    ("conv bias dropped",
     "for (long p = 0; p < hw; ++p) y[p] = b ? b[o] : 0.0;",
     "for (long p = 0; p < hw; ++p) y[p] = 0.0;",
     [(PINS.test_conv_linearity_and_bias, ())]),
    ("offset sign flipped",
     "x[p] = ((double)F[p] - offset) * gain * in_scale;",
     "x[p] = ((double)F[p] + offset) * gain * in_scale;",
     [(PINS.test_preprocess_closed_form, ())]),
    ("tie-break reversed",
     "if (!(v > nv || (v == nv && idx < nidx))) keep = 0;",
     "if (!(v > nv || (v == nv && idx > nidx))) keep = 0;",
     [(PINS.test_detect_exhaustive_3x3, ())]),
    ("residual dropped",
     "double s = a[k] + u[k];",
     "double s = u[k];",
     [(PINS.test_net_matches_torch_composition, ("A",))]),
    ("head bias dropped",
     "for (long k = 0; k < hw; ++k) m[k] = bd[q];",
     "for (long k = 0; k < hw; ++k) m[k] = 0.0;",
     [(UNC.test_head_closed_form, ("AU",))]),
    ("BF16 rounding truncates",
     "u += 0x7FFFu + lsb;",
     "u += 0u * lsb;",
     [(PINS.test_bf16_rounding_matches_torch, ())]),
    ("FP8 group exponent one too small",
     "int k = (e - 1) - (f <= 1.75 ? 8 : 7);",
     "int k = (e - 1) - (f <= 1.75 ? 9 : 8);",
     [(PINS.test_fp8_group_exponent_is_smallest_fitting_power_of_two, ())]),
    ("FP8 weight scale from the whole tensor's maximum",
     "for (long k = 0; k < per_out; ++k) if (fabs(wo[k]) > mx) mx = fabs(wo[k]);",
     "for (long k = 0; k < per_out * cout; ++k) if (fabs(W[k]) > mx) mx = fabs(W[k]);",
     [(FP8.test_fp8_weight_quant_closed_form, ()), (FP8.test_fp8_weight_quant_per_channel_properties, ())]),
    ("FP8 weights multiplied by the scale instead of its inverse",
     "float inv = (float)(448.0 / mx);",
     "float inv = (float)(mx / 448.0);",
     [(FP8.test_fp8_weight_quant_closed_form, ())]),
    ("FP8 stem output left unrounded",
     "if (quant == 2 && nblocks > 0) or_store_fp8_groups(a, C, hw);",
     ";",
     [(FP8.test_fp8_emulation_matches_torch_composition, (48, (1, 2, 4)))]),
    ("FP8 block intermediate left unrounded",
     "if (quant == 2) or_store_fp8_groups(t, C, hw);",
     ";",
     [(FP8.test_fp8_emulation_matches_torch_composition, (48, (1, 2, 4)))]),
    ("FP8 last block output rounded before the head",
     "if (quant == 2 && blk + 1 < nblocks) or_store_fp8_groups(a, C, hw);",
     "if (quant == 2) or_store_fp8_groups(a, C, hw);",
     [(FP8.test_fp8_emulation_matches_torch_composition, (48, (1, 2, 4)))]),
    ("split BF16: the wl xh term dropped",
     "    or_conv3x3(xh, cin, h, w, wl, NULL, cout, d, tmp);       /* Wl xh */\n    for (long k = 0; k < (long)cout * hw; ++k) out[k] += tmp[k];",
     "    or_conv3x3(xh, cin, h, w, wl, NULL, cout, d, tmp);       /* Wl xh */",
     [(B3.test_bf16x3_emulation_matches_torch_composition, (32, (1, 2, 4)))]),
    ("split BF16: lo taken without rounding",
     "        lo[k] = or_round_bf16(f - hi);",
     "        lo[k] = f - hi;",
     [(B3.test_split_matches_torch_casts_and_error_bound, ())]),
    ("split BF16: activations stored unrounded",
     "    if (quant == 3) return (double)(float)v;   /* split BF16 stores FP32 */",
     "    if (quant == 3) return v;",
     [(B3.test_bf16x3_emulation_matches_torch_composition, (32, (1, 2, 4)))]),
    ("dense layer reads one growth group too few",
     "            const int cin = C + i * G;",
     "            const int cin = C + (i > 0 ? i - 1 : 0) * G;",
     [(DN.test_dense_net_matches_torch_composition, (S.NET_D,))]),
    ("dense transition without ReLU",
     "        pointwise(cat, CT, hw, Wd, bd, C, 1, t);",
     "        pointwise(cat, CT, hw, Wd, bd, C, 0, t);",
     [(DN.test_dense_net_matches_torch_composition, (S.NET_D,))]),
    ("U-Net pooling reads one row of each window",
     "                for (int dy = 0; dy < 2; ++dy)",
     "                for (int dy = 0; dy < 1; ++dy)",
     [(DN.test_unet_matches_torch_composition, (DN.UNET_SMALL, 38, 29))]),
    ("U-Net upsampling takes the right neighbour",
     "out[((long)c * h + y) * w + x] = in[((long)c * h2 + y / 2) * w2 + x / 2];",
     "out[((long)c * h + y) * w + x] = in[((long)c * h2 + y / 2) * w2 + ((x + 1) / 2 < w2 ? (x + 1) / 2 : w2 - 1)];",
     [(DN.test_unet_matches_torch_composition, (DN.UNET_SMALL, 38, 29))]),
    ("U-Net skip and upsampled halves swapped",
     "    memcpy(c0, a0, sizeof(double) * C * n0);\n    up2(u1, C, h, w, c0 + C * n0);",
     "    memcpy(c0 + C * n0, a0, sizeof(double) * C * n0);\n    up2(u1, C, h, w, c0);",
     [(DN.test_unet_matches_torch_composition, (DN.UNET_SMALL, 38, 29))]),
    ("gate pool takes the last maximum",
     "if (h2[(long)c * hw + k] > h2[(long)c * hw + a]) a = k;",
     "if (h2[(long)c * hw + k] >= h2[(long)c * hw + a]) a = k;",
     [(PINS.test_gate_max_gradient_goes_to_first_maximum, ())]),
    ("camera gain and offset swapped",
     "x[p] = ((double)F[p] - offset[p]) * gain[p] * in_scale;",
     "x[p] = ((double)F[p] - gain[p]) * offset[p] * in_scale;",
     [(CAM.test_per_pixel_maps_equal_rescaled_frame, (S.make_net("A", 1),))]),
]


@pytest.mark.parametrize("name,old,new,pins", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_reject_a_planted_mistake(name, old, new, pins, tmp_path, monkeypatch):
    src = open(oracle._SRC).read()
    assert src.count(old) == 1, "the planted mistake's target text must occur once"
    mutant = tmp_path / "oracle_mutant.c"
    mutant.write_text(src.replace(old, new))
    lib = tmp_path / "liboracle_mutant.so"
    subprocess.check_call(["gcc", *oracle.GCC_FLAGS, str(mutant), "-o", str(lib), "-lm"])
    monkeypatch.setattr(oracle, "build", lambda force=False: str(lib))
    monkeypatch.setattr(oracle, "_lib", None)
    failed = []
    for pin, args in pins:
        try:
            pin(*args)
        except AssertionError:
            failed.append(pin.__name__)
    assert failed, f"no pin caught: {name}"


PY_MUTANTS = [
    ("pixel centre half dropped", "records",
     'out["x"] = cols + 0.5 + maps[1, rows, cols]',
     'out["x"] = cols + maps[1, rows, cols]',
     [(PINS.test_records_coordinates, ())]),
    ("x takes the y offset plane", "records",
     "cols + 0.5 + maps[1, rows, cols]",
     "cols + 0.5 + maps[2, rows, cols]",
     [(PINS.test_records_coordinates, ())]),
    ("softplus loses its small values", "softplus",
     "np.maximum(u, 0.0) + np.log1p(np.exp(-np.abs(u)))",
     "np.maximum(u, 0.0)",
     [(UNC.test_softplus_special_values, ())]),
    ("softplus in the overflowing form", "softplus",
     "np.maximum(u, 0.0) + np.log1p(np.exp(-np.abs(u)))",
     "np.log1p(np.exp(u))",
     [(UNC.test_softplus_special_values, ())]),
    ("background scaled the wrong way", "uncertainties",
     "sp[4] / spec.in_scale",
     "sp[4] * spec.in_scale",
     [(UNC.test_uncertainty_units_at_zero_raw_value, ())]),
    ("sigma filter reads the z plane", "sigma_filter",
     "(sigma_of(maps[6]) <= max_sigma_px)",
     "(sigma_of(maps[7]) <= max_sigma_px)",
     [(UNC.test_sigma_filter_invariants, ())]),
    ("threshold turned into a logit with the wrong odds", "localize",
     "math.log(threshold / (1.0 - threshold))",
     "math.log(threshold / (1.0 + threshold))",
     [(PINS.test_localize_threshold_is_a_probability, (0.3,))]),
    ("count variance without the (1 - p) factor", "train.frame_loss",
     "v = float(np.sum(p * (1 - p))) + VAR_EPS",
     "v = float(np.sum(p)) + VAR_EPS",
     [(TR.test_count_term_closed_form, ())]),
    ("mixture weights not divided by the expected count", "train.frame_loss",
     "logw = _log_sig(l) - math.log(mu)",
     "logw = _log_sig(l)",
     [(TR.test_loss_and_gradients_match_torch_autograd, ())]),
    ("sigma gradient without the softplus derivative", "train.frame_loss",
     "(tv[d] - mean[d]) ** 2 / s[d] ** 3) * _sig(maps[5 + d])",
     "(tv[d] - mean[d]) ** 2 / s[d] ** 3)",
     [(TR.test_loss_and_gradients_match_torch_autograd, ())]),
    ("transposed convolution left unflipped", "train._flip_t",
     "W[:, :, ::-1, ::-1].transpose(1, 0, 2, 3)",
     "W.transpose(1, 0, 2, 3)",
     [(TR.test_transposed_conv_is_the_adjoint, ())]),
    ("upsampling gradient takes one fine pixel instead of the sum", "train._up2_back",
     "return pad.reshape(C, h2, 2, w2, 2).sum(axis=(2, 4))",
     "return pad.reshape(C, h2, 2, w2, 2)[:, :, 0, :, 0]",
     [(TR.test_pooling_and_upsampling_gradients_are_adjoint, ())]),
    ("pooling gradient sent to the window's last maximum", "train._pool2",
     "return win.max(axis=-1), np.argmax(win, axis=-1)",
     "return win.max(axis=-1), 3 - np.argmax(win[..., ::-1], axis=-1)",
     [(TR.test_pooling_and_upsampling_gradients_are_adjoint, ())]),
    ("dense layer gradient without its ReLU mask", "train.dense_frame_grads",
     "gl = gc[lo:lo + Gr] * (cat[lo:lo + Gr] > 0)",
     "gl = gc[lo:lo + Gr]",
     [(TR.test_dense_loss_and_gradients_match_torch_autograd, ())]),
    ("dense layer's input gradient overwritten instead of added", "train.dense_frame_grads",
     "gc[:lo] += conv3x3(gl, _flip_t(W[f\"blk{k}.l{i}.w\"]), None, d)",
     "gc[:lo] = conv3x3(gl, _flip_t(W[f\"blk{k}.l{i}.w\"]), None, d)",
     [(TR.test_dense_loss_and_gradients_match_torch_autograd, ())]),
]


@pytest.mark.parametrize("name,fname,old,new,pins", PY_MUTANTS, ids=[m[0] for m in PY_MUTANTS])
def test_pins_reject_a_planted_python_mistake(name, fname, old, new, pins, monkeypatch):
    mod = oracle
    if fname.startswith("train."):
        mod, fname = oracle.train, fname.split(".", 1)[1]
    src = textwrap.dedent(inspect.getsource(getattr(mod, fname)))
    assert src.count(old) == 1, "the planted mistake's target text must occur once"
    ns = dict(vars(mod))
    exec(compile(src.replace(old, new), f"<planted mistake in {mod.__name__}.{fname}>", "exec"), ns)
    monkeypatch.setattr(mod, fname, ns[fname])
    failed = []
    with np.errstate(all="ignore"):
        for pin, args in pins:
            try:
                pin(*args)
            except AssertionError:
                failed.append(pin.__name__)
    assert failed, f"no pin caught: {name}"
