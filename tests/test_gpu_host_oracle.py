"""The host-memory entry points against the FP64 oracle directly (paper
Sec. 2.2: frames preloaded in host memory, copied to the device while the
previous batch is inferred, only coordinates returned to the host).

dl_localize (copy in, localize, copy the records out), dl_localize_pipelined
with the overlap on and off and with pageable and pinned frames, and the
variants with uncertainties (dl_localize_unc, dl_localize_pipelined_unc): each
returns the oracle's emitters (outside the pixels whose decision FP32 rounding
may flip), in (frame, row, col) order with frame indices running over all
batches, and every record field within the bound the FP32 map tolerance
implies.  The last test orders two device-path runs queued on different
streams with no synchronisation between them.
"""
import ctypes

import numpy as np
import pytest

import oracle
import smlm_synth as S
from tests.parity import compare_emitters, record_field_errors

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no HIP device", allow_module_level=True)
import paper_2410_02314_amd as dl  # noqa: E402
from tests.test_gpu_fp32 import gpu_localize  # noqa: E402

DEV = torch.device("cuda:0")


def _check(rec, ref, ref_maps, spec):
    cmp = compare_emitters(rec, ref, ref_maps)
    assert cmp["non_exempt_mismatch"] == 0 and cmp["order_ok"], cmp
    assert cmp["matched"] > 0.95 * len(ref) and len(ref) > 50
    err = record_field_errors(rec, ref, ref_maps, spec)
    print(cmp["matched"], err)
    for k in ("x", "y", "z", "photons", "prob"):
        assert err[k] <= 1.0, (k, err)


def _pinned_copy(frames):
    p = dl.host_alloc(frames.nbytes)
    buf = (ctypes.c_char * frames.nbytes).from_address(p)
    arr = np.frombuffer(buf, dtype=np.uint16).reshape(frames.shape)
    arr[...] = frames
    return p, arr


@pytest.fixture(scope="module")
def net_b_small():
    """Net B (non-zero z rows), 3 batches of 2 ragged frames, oracle records."""
    spec, w = S.make_net("B", 2)
    frames = S.render_frames(6, 96, 136, "full", 71)
    ref, ref_maps = oracle.localize(frames, spec, w, return_maps=True)
    return spec, w, frames, ref, ref_maps


def test_dl_localize_matches_oracle(net_b_small):
    spec, w, frames, ref, ref_maps = net_b_small
    net = dl.Net(S.serialize_weights(spec, w))
    rec = net.localize(frames)
    assert np.any(np.abs(ref["z"]) > 50)            # the z field is really exercised
    _check(rec, ref, ref_maps, spec)


@pytest.mark.parametrize("pinned", [False, True])
@pytest.mark.parametrize("overlap", [True, False])
def test_dl_localize_pipelined_matches_oracle(net_b_small, pinned, overlap):
    spec, w, frames, ref, ref_maps = net_b_small
    net = dl.Net(S.serialize_weights(spec, w))
    batches = frames.reshape(3, 2, *frames.shape[1:])
    p = None
    if pinned:
        p, batches = _pinned_copy(batches)
    try:
        rec = net.localize_pipelined(batches, overlap=overlap)
    finally:
        if p:
            dl.host_free(p)
    _check(rec, ref, ref_maps, spec)


@pytest.mark.parametrize("pipelined", [False, True])
def test_host_uncertainty_entry_points_match_oracle(pipelined):
    spec, w = S.make_net("AU", 1)
    frames = S.render_frames(4, 128, 120, "tiny", 72)
    ref, ref_unc, ref_maps = oracle.localize(frames, spec, w, return_maps=True, with_uncertainty=True)
    net = dl.Net(S.serialize_weights(spec, w))
    if pipelined:
        rec, unc = net.localize_pipelined_unc(frames.reshape(2, 2, 128, 120), overlap=True)
    else:
        rec, unc = net.localize_unc(frames)
    _check(rec, ref, ref_maps, spec)
    gk = {(int(a), int(b), int(c)): i for i, (a, b, c) in enumerate(zip(rec["frame"], rec["row"], rec["col"]))}
    rk = {(int(a), int(b), int(c)): i for i, (a, b, c) in enumerate(zip(ref["frame"], ref["row"], ref["col"]))}
    both = [k for k in gk if k in rk]
    gi = np.array([gk[k] for k in both])
    ri = np.array([rk[k] for k in both])
    # softplus is 1-Lipschitz: each uncertainty's error is at most its raw
    # plane's, 1e-4 (|u| + rms u) times the unit
    units = {"sigma_x_px": ("sigma_x", 5, 1.0), "sigma_y_px": ("sigma_y", 6, 1.0),
             "sigma_z_nm": ("sigma_z", 7, spec.z_scale), "sigma_photons": ("sigma_photons", 8, spec.ph_scale),
             "background": ("background", 9, 1.0 / spec.in_scale)}
    fr = np.array([k[0] for k in both])
    rows = np.array([k[1] for k in both])
    cols = np.array([k[2] for k in both])
    for g_name, (o_name, plane, unit) in units.items():
        u = ref_maps[fr, plane, rows, cols]
        rms = np.sqrt(np.mean(ref_maps[:, plane] ** 2, axis=(1, 2)))[fr]
        bound = 1e-4 * (np.abs(u) + rms) * unit + 1e-6 * (1 + np.abs(ref_unc[o_name][ri]))
        assert np.all(np.abs(unc[g_name][gi] - ref_unc[o_name][ri]) <= bound), g_name


def test_runs_on_two_streams_are_ordered():
    """Two device-path runs on two streams, no synchronisation between them:
    they share the handle's workspace, so the second waits for the first on
    the device and both equal their serial results."""
    spec, w = S.make_net("B", 2)
    net = dl.Net(S.serialize_weights(spec, w), precision="bf16")
    fa = S.render_frames(2, 512, 512, "full", 81)
    fb = S.render_frames(2, 512, 512, "full", 82)
    ra, _ = gpu_localize(net, fa)
    rb, _ = gpu_localize(net, fb)
    cap = 2 * 512 * 512 // 8
    da = torch.from_numpy(fa).to(DEV)
    db = torch.from_numpy(fb).to(DEV)
    outs = [torch.zeros((cap, 8), dtype=torch.int32, device=DEV) for _ in range(2)]
    cnts = [torch.full((3,), -1, dtype=torch.int32, device=DEV) for _ in range(2)]
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    for _ in range(3):
        net.localize_device(da, outs[0], cnts[0], s1)
        net.localize_device(db, outs[1], cnts[1], s2)
    torch.cuda.synchronize()
    ga = dl.emitters_from_device(outs[0], int(cnts[0][2].item()))
    gb = dl.emitters_from_device(outs[1], int(cnts[1][2].item()))
    assert np.array_equal(ga, ra) and np.array_equal(gb, rb)
