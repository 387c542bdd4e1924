"""GPU training of the localisation network (Sec. 3.3: DECODE's count and
localisation loss with the binary cross-entropy on the detection probability)
against the FP64 training oracle, through the C ABI.

* dl_train_grad: the three loss terms and the gradient of every weight tensor
  of the residual network with the 10-output head (C = 32 and 16), within
  1e-4 relative (L2 per tensor, FP32 against FP64), on batches with a frame
  without emitters, ragged widths and tall frames that give the weight
  gradient's waves several rows; the same bits on a second call;
* dl_train_step: one step equals the oracle's Adam step on the oracle's
  gradient; forty steps lower the loss; the inference path then runs the
  trained weights (its maps equal the oracle's on dl_get_params' weights);
* the dense-connection network (backward through the concatenation and the
  fused 1x1 transition) and with the two-stage U-Net (max pooling and
  upsampling gradients, skip concatenations): gradients against the oracle
  for several widths, depths, dilations and odd sizes, nets DT and DU with
  the 10-output head, a tall frame; an Adam step and the trained weights in
  the inference path;
* training improves localisation: 500 steps from net AU's initial weights
  raise recall and precision and lower the lateral error against the ground
  truth on held-out frames;
* refusals: nets the training kernels do not cover.
"""
import numpy as np
import pytest

import oracle
import oracle.train as T
import smlm_synth as S
from tests.parity import map_rel_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no HIP device", allow_module_level=True)
import paper_2410_02314_amd as dl  # noqa: E402

DEV = torch.device("cuda:0")
TOL = 1e-4


def batch(n, h, w, seed, empty_last=True):
    frames, truths = S.render_frames(n, h, w, "tiny", seed, with_truth=True)
    truths = [S.truth_array(t, h, w) for t in truths]
    if empty_last:
        frames[-1] = 100
        truths[-1] = truths[-1][:0]
    return frames, truths


def device_truth(truths):
    off = np.zeros(len(truths) + 1, np.int32)
    rows = []
    for f, t in enumerate(truths):
        off[f + 1] = off[f] + len(t)
        rows += [[r["x"], r["y"], r["z_nm"], r["photons"]] for r in t]
    tr = np.asarray(rows, np.float32).reshape(-1, 4)
    return torch.from_numpy(tr).to(DEV), torch.from_numpy(off).to(DEV)


def net_and_weights(spec, seed):
    w = S.he_normal_weights(spec, seed, bias_std=0.05)
    w["head.w"] = (w["head.w"] * 0.3).astype(np.float32)
    return w, dl.Net(S.serialize_weights(spec, w))


def gpu_grads(net, spec, frames, truths):
    fr = torch.from_numpy(frames).to(DEV)
    tr, off = device_truth(truths)
    grad = torch.full((net.nparams,), float("nan"), dtype=torch.float32, device=DEV)
    loss = net.train_grad(fr, tr, off, grad)
    torch.cuda.synchronize()
    return loss.cpu().numpy(), S.unflat_weights(spec, grad.cpu().numpy())


# the weight-gradient kernel gives each wave ceil(n h / 2048) rows: the two tall
# single frames run two rows per wave and end on a wave with one row of an odd
# number of steps (7 pixel pairs for C = 32, 3 pixel quads for C = 16); the
# 2201 x 13 frame holds more than 256 true emitters (two emitter groups in the
# log-sum-exp) and its log-sum-exp chunks span two 256-pixel groups
@pytest.mark.parametrize("spec,n,h,w", [(S.NetSpec("t32", 32, (1, 2), head_outputs=10), 3, 40, 52),
                                        (S.NetSpec("t16", 16, (1, 3, 2), head_outputs=10), 2, 33, 70),
                                        (S.NET_AU, 2, 64, 64),
                                        (S.NetSpec("t32", 32, (1, 2), head_outputs=10), 1, 2201, 13),
                                        (S.NetSpec("t16", 16, (2, 1), head_outputs=10), 1, 2059, 9)])
def test_gradients_match_the_oracle(spec, n, h, w):
    wts, net = net_and_weights(spec, 11)
    frames, truths = batch(n, h, w, 21, empty_last=n > 1)
    L, G = T.batch_grads(frames, truths, spec, wts)
    loss, g = gpu_grads(net, spec, frames, truths)
    print(spec.name, L, loss)
    for i, k in enumerate(["total", "bce", "count", "loc"]):
        assert abs(loss[i] - L[k]) <= TOL * (abs(L[k]) + 1e-3), (k, loss[i], L[k])
    for k in G:
        ref = np.asarray(G[k])
        err = np.linalg.norm(g[k] - ref) / (np.linalg.norm(ref) + 1e-30)
        print(k, err)
        assert np.isfinite(g[k]).all() and err <= TOL, (k, err)
    loss2, g2 = gpu_grads(net, spec, frames, truths)
    assert np.array_equal(loss, loss2) and all(np.array_equal(g[k], g2[k]) for k in g)


def test_adam_step_matches_the_oracle_and_training_lowers_the_loss():
    spec = S.NET_AU
    wts, net = net_and_weights(spec, 12)
    frames, truths = batch(4, 64, 64, 22, empty_last=False)
    fr = torch.from_numpy(frames).to(DEV)
    tr, off = device_truth(truths)
    # one step against the oracle's Adam on the oracle's gradient
    _, G = T.batch_grads(frames, truths, spec, wts)
    theta = S.flat_weights(spec, wts).astype(np.float64)
    m, v = np.zeros_like(theta), np.zeros_like(theta)
    lr = 1e-3
    oracle.adam_step(theta, m, v, S.flat_weights(spec, {k: np.asarray(g) for k, g in G.items()}).astype(np.float64), 1,
                     lr=lr)
    net.train_step(fr, tr, off, lr)
    got = net.get_params()
    # the step moves each weight by about lr; FP32 gradients near zero may flip
    # a step's sign, so compare the moved amounts
    moved = got.astype(np.float64) - S.flat_weights(spec, wts)
    ref_moved = theta - S.flat_weights(spec, wts)
    assert np.mean(np.abs(moved - ref_moved) <= 1e-6 + 1e-3 * np.abs(ref_moved)) >= 0.99
    # training lowers the loss
    losses = []
    for _ in range(40):
        losses.append(float(net.train_step(fr, tr, off, 1e-3).cpu()[0]))
    print(losses[:3], losses[-3:])
    assert losses[-1] < losses[0]
    # the inference path runs the trained weights
    p = net.get_params()
    tw = S.unflat_weights(spec, p)
    maps = torch.empty((4, 10, 64, 64), dtype=torch.float32, device=DEV)
    net.maps_device(fr, maps)
    torch.cuda.synchronize()
    ref = oracle.net_maps_batch(frames, spec, tw)
    assert map_rel_err(maps.cpu().numpy(), ref).max() <= TOL


# the dense-connection network: C = 32 with four layers (CT = 96), C = 32 with
# three (CT = 80: the transition's weight gradient in 16-row pieces), C = 16,
# net DT itself (dilations 2 .. 16), and a tall frame (two rows per wave)
@pytest.mark.parametrize("spec,n,h,w", [(S.DenseSpec("td4", 32, (2, 4), head_outputs=10), 2, 40, 52),
                                        (S.DenseSpec("td3", 32, (1, 3), layers=3, head_outputs=10), 2, 37, 45),
                                        (S.DenseSpec("td16", 16, (1, 2), layers=2, head_outputs=10), 2, 33, 70),
                                        (S.NET_DT, 1, 64, 64),
                                        (S.DenseSpec("td2", 32, (2,), layers=2, head_outputs=10), 1, 2201, 13),
                                        # with the two-stage U-Net: even and odd sizes (partial pooling
                                        # windows at both levels), C = 16, net DU with the 10-output head
                                        (S.DenseSpec("tu", 32, (2,), layers=2, head_outputs=10, unet=2), 2, 40, 52),
                                        (S.DenseSpec("tu", 32, (1, 2), layers=2, head_outputs=10, unet=2), 2, 37, 45),
                                        (S.DenseSpec("tu16", 16, (2,), layers=3, head_outputs=10, unet=2), 1, 33, 70),
                                        (S.NET_DUT, 1, 64, 64)])
def test_dense_gradients_match_the_oracle(spec, n, h, w):
    wts, net = net_and_weights(spec, 13)
    frames, truths = batch(n, h, w, 23, empty_last=n > 1)
    L, G = T.batch_grads(frames, truths, spec, wts)
    loss, g = gpu_grads(net, spec, frames, truths)
    print(spec.name, L, loss)
    for i, k in enumerate(["total", "bce", "count", "loc"]):
        assert abs(loss[i] - L[k]) <= TOL * (abs(L[k]) + 1e-3), (k, loss[i], L[k])
    assert set(g) == set(G)
    for k in G:
        ref = np.asarray(G[k])
        err = np.linalg.norm(g[k] - ref) / (np.linalg.norm(ref) + 1e-30)
        print(k, err)
        assert np.isfinite(g[k]).all() and err <= TOL, (k, err)
    loss2, g2 = gpu_grads(net, spec, frames, truths)
    assert np.array_equal(loss, loss2) and all(np.array_equal(g[k], g2[k]) for k in g)


@pytest.mark.parametrize("spec", [S.DenseSpec("td4", 32, (2, 4), head_outputs=10),
                                  S.DenseSpec("tu", 32, (2, 4), layers=2, head_outputs=10, unet=2)])
def test_dense_adam_step_and_the_trained_weights_in_inference(spec):
    wts, net = net_and_weights(spec, 14)
    frames, truths = batch(4, 48, 48, 24, empty_last=False)
    fr = torch.from_numpy(frames).to(DEV)
    tr, off = device_truth(truths)
    _, G = T.batch_grads(frames, truths, spec, wts)
    theta = S.flat_weights(spec, wts).astype(np.float64)
    m, v = np.zeros_like(theta), np.zeros_like(theta)
    oracle.adam_step(theta, m, v, S.flat_weights(spec, {k: np.asarray(g) for k, g in G.items()}).astype(np.float64), 1,
                     lr=1e-3)
    net.train_step(fr, tr, off, 1e-3)
    moved = net.get_params().astype(np.float64) - S.flat_weights(spec, wts)
    ref_moved = theta - S.flat_weights(spec, wts)
    assert np.mean(np.abs(moved - ref_moved) <= 1e-6 + 1e-3 * np.abs(ref_moved)) >= 0.99
    losses = [float(net.train_step(fr, tr, off, 1e-3).cpu()[0]) for _ in range(30)]
    print(losses[:3], losses[-3:])
    assert losses[-1] < losses[0]
    tw = S.unflat_weights(spec, net.get_params())
    maps = torch.empty((4, 10, 48, 48), dtype=torch.float32, device=DEV)
    net.maps_device(fr, maps)
    torch.cuda.synchronize()
    ref = oracle.net_maps_batch(frames, spec, tw)
    assert map_rel_err(maps.cpu().numpy(), ref).max() <= TOL


@pytest.mark.parametrize("spec", [S.NetSpec("t32", 32, (1, 2), head_outputs=10),
                                  S.DenseSpec("td", 32, (2,), layers=2, head_outputs=10),
                                  S.DenseSpec("tu", 16, (1,), layers=2, head_outputs=10, unet=2)])
@pytest.mark.parametrize("n,h,w,no_emitters", [(2, 5, 3, False), (1, 7, 1, False), (3, 9, 11, True)])
def test_tiny_frames_and_batches_without_emitters(spec, n, h, w, no_emitters):
    """Frames narrower than one MFMA step and shorter than a conv tile (1-pixel
    U-Net levels), and a batch whose frames hold no true emitter (the
    localisation term vanishes)."""
    wts, net = net_and_weights(spec, 15)
    frames, truths = S.render_frames(n, h, w, "tiny", 25, with_truth=True)
    truths = [S.truth_array(t, h, w) for t in truths]
    if no_emitters:
        truths = [t[:0] for t in truths]
    else:                                # one planted target per frame (frames this small hold no rendered one)
        for f in range(n):
            t = np.zeros(1, S.TRUTH_DTYPE)
            t["x"], t["y"], t["z_nm"], t["photons"] = 0.37 * w + 0.1 * f, 0.61 * h, 120.0 - 40 * f, 2500.0
            truths[f] = t
    L, G = T.batch_grads(frames, truths, spec, wts)
    loss, g = gpu_grads(net, spec, frames, truths)
    if no_emitters:
        assert loss[3] == 0.0
    for i, k in enumerate(["total", "bce", "count", "loc"]):
        assert abs(loss[i] - L[k]) <= TOL * (abs(L[k]) + 1e-3), (k, loss[i], L[k])
    for k in G:
        ref = np.asarray(G[k])
        err = np.linalg.norm(g[k] - ref) / (np.linalg.norm(ref) + 1e-30)
        assert np.isfinite(g[k]).all() and err <= TOL, (k, err)


def test_training_teaches_the_net_to_localise():
    """500 Adam steps from net AU's initial weights on 64 synthetic frames: on
    8 held-out frames the emitter list matches the ground truth (within 1 px)
    with higher recall and precision and a smaller lateral error than before
    training, and the loss stays finite (the sigma floor bounds the mixture's
    likelihood; without it this run went NaN at step 82)."""
    import bench_workloads as BW
    spec, w = S.make_net("AU", 1)
    r = BW.train_eval(S, spec, w, steps=500)
    print(r)
    b, a = r["before"], r["after"]
    assert np.isfinite(r["loss_after"])
    assert a["recall"] >= b["recall"] + 0.1 and a["recall"] >= 0.8
    assert a["precision"] >= 0.95 and a["precision"] > b["precision"]
    assert a["rms_xy_px"] <= 0.25 and a["rms_xy_px"] < b["rms_xy_px"]


def test_nets_the_training_kernels_do_not_cover_are_refused():
    fr = torch.from_numpy(S.render_frames(1, 32, 32, "tiny", 3)).to(DEV)
    tr = torch.zeros((0, 4), dtype=torch.float32, device=DEV)
    off = torch.zeros(2, dtype=torch.int32, device=DEV)
    for name in ("B", "BU", "A", "D"):           # C = 48, a 5-output head
        spec, w = S.make_net(name, 2 if name[0] == "B" else 1 if name == "A" else 3)
        net = dl.Net(S.serialize_weights(spec, w))
        with pytest.raises(dl.DlocError) as e:
            net.train_grad(fr, tr, off)
        assert e.value.code == dl.DL_ERR_UNSUPPORTED, name
    # a dense net with a growth other than 16
    for spec in (S.DenseSpec("dg32", 32, (2,), growth=32, head_outputs=10),):
        net = dl.Net(S.serialize_weights(spec, S.he_normal_weights(spec, 1)))
        with pytest.raises(dl.DlocError) as e:
            net.train_grad(fr, tr, off)
        assert e.value.code == dl.DL_ERR_UNSUPPORTED, spec.name
    # a frame row wider than the weight-gradient kernels' 32-bit row offsets
    # cover (refused before any work is queued)
    spec, w = S.make_net("AU", 1)
    net = dl.Net(S.serialize_weights(spec, w))
    wide = torch.from_numpy(np.zeros((1, 1, (1 << 20) + 64), np.uint16)).to(DEV)
    with pytest.raises(dl.DlocError) as e:
        net.train_grad(wide, tr, off)
    assert e.value.code == dl.DL_ERR_UNSUPPORTED and "2^20" in str(e.value)
