"""Pins of the training oracle (``oracle.train``): the loss of Sec. 3.3 (binary
cross-entropy on the detection probability together with DECODE's count and
localisation terms) and the gradients of every weight of the residual network
with the 10-output head.

* the loss and every gradient against an independent torch float64
  composition differentiated by autograd (conv2d with dilation, logsigmoid,
  softplus, logsumexp), on frames with emitters, one frame without;
* central finite differences of the whole loss for sampled weights;
* closed forms: the count term at p = 1/2 everywhere; the localisation term
  when one pixel holds all the probability (a Gaussian's negative
  log-likelihood); the cross-entropy term on a known occupancy;
* the transposed convolution the backward pass uses against the adjoint
  identity <conv(x), y> = <x, conv_T(y)>;
* the dense-connection network (backward through the concatenation and the
  1x1 transition): loss and gradients against torch autograd of a composition
  from torch.cat and conv2d, finite differences, and its forward maps against
  the inference oracle.
"""
import math

import numpy as np
import pytest

import oracle
import oracle.train as T
import smlm_synth as S

torch = pytest.importorskip("torch")
F = torch.nn.functional

SPEC = S.NetSpec("t16", 16, (1, 2), head_outputs=10)


def data(n=2, h=24, w=28, seed=5, empty_last=True):
    frames, truths = S.render_frames(n, h, w, "tiny", seed, with_truth=True)
    truths = [S.truth_array(t, h, w) for t in truths]
    if empty_last:
        frames[-1] = 100
        truths[-1] = truths[-1][:0]
    return frames, truths


def weights(seed=3):
    w = S.he_normal_weights(SPEC, seed, bias_std=0.05)
    w["head.w"] = (w["head.w"] * 0.3).astype(np.float32)
    return w


def torch_loss(frames, truths, spec, wts, gain=0.5, offset=100.0):
    P = {k: torch.tensor(np.asarray(v, np.float64), requires_grad=True) for k, v in wts.items()}
    total = 0.0
    for f in range(len(frames)):
        x = (torch.from_numpy(frames[f].astype(np.float64)) - offset) * gain * spec.in_scale
        a = F.relu(F.conv2d(x[None, None], P["stem.w"], P["stem.b"], padding=1))
        for k, d in enumerate(spec.dilations):
            t = F.relu(F.conv2d(a, P[f"blk{k}.w1"], P[f"blk{k}.b1"], padding=d, dilation=d))
            a = F.relu(F.conv2d(t, P[f"blk{k}.w2"], P[f"blk{k}.b2"], padding=d, dilation=d) + a)
        m = F.conv2d(a, P["head.w"][:, :, None, None], P["head.b"])[0]
        h, w = m.shape[1:]
        l = m[0]
        p = torch.sigmoid(l)
        y = torch.zeros(h, w, dtype=torch.float64)
        for t in truths[f]:
            y[int(math.floor(t["y"])), int(math.floor(t["x"]))] = 1.0
        L = (F.softplus(l) - y * l).mean()
        E = len(truths[f])
        mu = p.sum()
        v = (p * (1 - p)).sum() + T.VAR_EPS
        L = L + 0.5 * torch.log(2 * math.pi * v) + (E - mu) ** 2 / (2 * v)
        rows, cols = torch.meshgrid(torch.arange(h, dtype=torch.float64), torch.arange(w, dtype=torch.float64),
                                    indexing="ij")
        mean = [cols + 0.5 + m[1], rows + 0.5 + m[2], m[3], m[4]]
        sd = [F.softplus(m[5 + d]) + 0.01 for d in range(4)]
        for t in truths[f]:
            tv = [t["x"], t["y"], t["z_nm"] / spec.z_scale, t["photons"] / spec.ph_scale]
            q = F.logsigmoid(l) - torch.log(mu)
            for d in range(4):
                q = q + torch.distributions.Normal(mean[d], sd[d]).log_prob(torch.tensor(float(tv[d]), dtype=torch.float64))
            L = L - torch.logsumexp(q.reshape(-1), 0)
        total = total + L
    total = total / len(frames)
    total.backward()
    return float(total.detach()), {k: v.grad.numpy() for k, v in P.items()}


DSPEC = S.DenseSpec("td", 16, (1, 2), layers=2, growth=16, head_outputs=10)


def dense_weights(seed=3):
    w = S.he_normal_weights(DSPEC, seed, bias_std=0.05)
    w["head.w"] = (w["head.w"] * 0.3).astype(np.float32)
    return w


def torch_dense_loss(frames, truths, spec, wts, gain=0.5, offset=100.0):
    """The dense-connection network and the same loss, composed from torch
    ops (cat over channels, conv2d with dilation, a 1x1 conv2d) and
    differentiated by autograd."""
    P = {k: torch.tensor(np.asarray(v, np.float64), requires_grad=True) for k, v in wts.items()}
    total = 0.0
    for f in range(len(frames)):
        x = (torch.from_numpy(frames[f].astype(np.float64)) - offset) * gain * spec.in_scale
        a = F.relu(F.conv2d(x[None, None], P["stem.w"], P["stem.b"], padding=1))
        for k, d in enumerate(spec.dilations):
            feats = [a]
            for i in range(spec.layers):
                inp = torch.cat(feats, dim=1)
                feats.append(F.relu(F.conv2d(inp, P[f"blk{k}.l{i}.w"], P[f"blk{k}.l{i}.b"], padding=d, dilation=d)))
            a = F.relu(F.conv2d(torch.cat(feats, dim=1), P[f"blk{k}.t.w"][:, :, None, None], P[f"blk{k}.t.b"]))
        m = F.conv2d(a, P["head.w"][:, :, None, None], P["head.b"])[0]
        total = total + _torch_frame_loss(m, truths[f], spec)
    total = total / len(frames)
    total.backward()
    return float(total.detach()), {k: v.grad.numpy() for k, v in P.items()}


def _torch_frame_loss(m, truth, spec):
    h, w = m.shape[1:]
    l = m[0]
    p = torch.sigmoid(l)
    y = torch.zeros(h, w, dtype=torch.float64)
    for t in truth:
        y[int(math.floor(t["y"])), int(math.floor(t["x"]))] = 1.0
    L = (F.softplus(l) - y * l).mean()
    E = len(truth)
    mu = p.sum()
    v = (p * (1 - p)).sum() + T.VAR_EPS
    L = L + 0.5 * torch.log(2 * math.pi * v) + (E - mu) ** 2 / (2 * v)
    rows, cols = torch.meshgrid(torch.arange(h, dtype=torch.float64), torch.arange(w, dtype=torch.float64),
                                indexing="ij")
    mean = [cols + 0.5 + m[1], rows + 0.5 + m[2], m[3], m[4]]
    sd = [F.softplus(m[5 + d]) + 0.01 for d in range(4)]
    for t in truth:
        tv = [t["x"], t["y"], t["z_nm"] / spec.z_scale, t["photons"] / spec.ph_scale]
        q = F.logsigmoid(l) - torch.log(mu)
        for d in range(4):
            q = q + torch.distributions.Normal(mean[d], sd[d]).log_prob(torch.tensor(float(tv[d]), dtype=torch.float64))
        L = L - torch.logsumexp(q.reshape(-1), 0)
    return L


def test_dense_loss_and_gradients_match_torch_autograd():
    frames, truths = data()
    wts = dense_weights()
    assert len(truths[0]) >= 2
    L, G = T.batch_grads(frames, truths, DSPEC, wts)
    Lt, Gt = torch_dense_loss(frames, truths, DSPEC, wts)
    assert set(G) == set(Gt)
    assert abs(L["total"] - Lt) <= 1e-10 * abs(Lt)
    for k in G:
        ref = Gt[k]
        err = np.linalg.norm(G[k] - ref) / (np.linalg.norm(ref) + 1e-300)
        assert err <= 1e-9, (k, err)


USPEC = S.DenseSpec("tu", 16, (1,), layers=2, growth=16, head_outputs=10, unet=2)


def torch_unet_loss(frames, truths, spec, wts, gain=0.5, offset=100.0):
    """The dense network with the two-stage U-Net, composed from torch ops:
    max_pool2d with ceil_mode (a window at an odd edge holds what it has),
    nearest interpolation cropped to the level, cat, conv2d."""
    P = {k: torch.tensor(np.asarray(v, np.float64), requires_grad=True) for k, v in wts.items()}
    total = 0.0
    for f in range(len(frames)):
        x = (torch.from_numpy(frames[f].astype(np.float64)) - offset) * gain * spec.in_scale
        a = F.relu(F.conv2d(x[None, None], P["stem.w"], P["stem.b"], padding=1))
        for k, d in enumerate(spec.dilations):
            feats = [a]
            for i in range(spec.layers):
                feats.append(F.relu(F.conv2d(torch.cat(feats, dim=1), P[f"blk{k}.l{i}.w"], P[f"blk{k}.l{i}.b"],
                                             padding=d, dilation=d)))
            a = F.relu(F.conv2d(torch.cat(feats, dim=1), P[f"blk{k}.t.w"][:, :, None, None], P[f"blk{k}.t.b"]))
        h, w = a.shape[2:]
        d1 = F.relu(F.conv2d(F.max_pool2d(a, 2, ceil_mode=True), P["unet.d1.w"], P["unet.d1.b"], padding=1))
        d2 = F.relu(F.conv2d(F.max_pool2d(d1, 2, ceil_mode=True), P["unet.d2.w"], P["unet.d2.b"], padding=1))
        up = F.interpolate(d2, scale_factor=2, mode="nearest")[:, :, :d1.shape[2], :d1.shape[3]]
        u1 = F.relu(F.conv2d(torch.cat([d1, up], dim=1), P["unet.u1.w"], P["unet.u1.b"], padding=1))
        up = F.interpolate(u1, scale_factor=2, mode="nearest")[:, :, :h, :w]
        u0 = F.relu(F.conv2d(torch.cat([a, up], dim=1), P["unet.u0.w"], P["unet.u0.b"], padding=1))
        m = F.conv2d(u0, P["head.w"][:, :, None, None], P["head.b"])[0]
        total = total + _torch_frame_loss(m, truths[f], spec)
    total = total / len(frames)
    total.backward()
    return float(total.detach()), {k: v.grad.numpy() for k, v in P.items()}


@pytest.mark.parametrize("h,w", [(24, 28), (23, 29)])
def test_unet_loss_and_gradients_match_torch_autograd(h, w):
    """Even and odd frame sizes (partial pooling windows at both levels)."""
    frames, truths = data(h=h, w=w)
    wts = S.he_normal_weights(USPEC, 6, bias_std=0.05)
    wts["head.w"] = (wts["head.w"] * 0.3).astype(np.float32)
    L, G = T.batch_grads(frames, truths, USPEC, wts)
    Lt, Gt = torch_unet_loss(frames, truths, USPEC, wts)
    assert set(G) == set(Gt)
    assert abs(L["total"] - Lt) <= 1e-10 * abs(Lt)
    for k in G:
        ref = Gt[k]
        err = np.linalg.norm(G[k] - ref) / (np.linalg.norm(ref) + 1e-300)
        assert err <= 1e-9, (k, err)
    # the training oracle's maps are the inference oracle's
    _, _, maps = T.dense_frame_grads(frames[0], truths[0], USPEC, wts)
    ref = oracle.net_maps(frames[0], USPEC, wts)
    assert np.max(np.abs(maps - ref)) <= 1e-12 * (1 + np.max(np.abs(ref)))


def test_pooling_and_upsampling_gradients_are_adjoint():
    """<pool(a) routed by argmax> and <up(v), g> = <v, up_back(g)> identities,
    and a tie routed to the window's first maximum."""
    r = np.random.default_rng(4)
    for h, w in ((6, 8), (7, 5)):
        v = r.standard_normal((3, (h + 1) // 2, (w + 1) // 2))
        g = r.standard_normal((3, h, w))
        assert abs(np.sum(T._up2(v, h, w) * g) - np.sum(v * T._up2_back(g, *v.shape[1:]))) <= 1e-12
        a = r.standard_normal((3, h, w))
        p, idx = T._pool2(a)
        gp = r.standard_normal(p.shape)
        back = T._pool2_back(gp, idx, h, w)
        # each window's gradient lands on a pixel holding the window's maximum
        assert abs(np.sum(back * a) - np.sum(gp * p)) <= 1e-12
        assert np.count_nonzero(back) == gp.size
    a = np.zeros((1, 2, 2))
    a[0, 1, 0] = a[0, 1, 1] = 5.0
    _, idx = T._pool2(a)
    assert T._pool2_back(np.ones((1, 1, 1)), idx, 2, 2)[0].tolist() == [[0.0, 0.0], [1.0, 0.0]]


def test_dense_finite_differences():
    frames, truths = data(n=1, empty_last=False)
    wts = dense_weights(4)
    _, G = T.batch_grads(frames, truths, DSPEC, wts)
    r = np.random.default_rng(8)
    for name in ["stem.w", "blk0.l0.w", "blk0.l1.w", "blk1.l1.b", "blk0.t.w", "blk1.t.b", "head.w"]:
        for _ in range(2):
            idx = tuple(int(r.integers(0, s)) for s in wts[name].shape)
            h = 1e-5
            wp = {k: np.asarray(v, np.float64).copy() for k, v in wts.items()}
            wm = {k: np.asarray(v, np.float64).copy() for k, v in wts.items()}
            wp[name][idx] += h
            wm[name][idx] -= h
            Lp, _ = T.batch_grads(frames, truths, DSPEC, wp)
            Lm, _ = T.batch_grads(frames, truths, DSPEC, wm)
            fd = (Lp["total"] - Lm["total"]) / (2 * h)
            assert abs(fd - G[name][idx]) <= 1e-5 * (abs(fd) + 1e-3), (name, idx, fd, G[name][idx])


def test_dense_forward_matches_the_inference_oracle():
    """The training oracle's maps are the inference oracle's (its C code)."""
    frames, _ = data(n=1, empty_last=False)
    wts = dense_weights(5)
    _, _, maps = T.dense_frame_grads(frames[0], np.zeros(0, S.TRUTH_DTYPE), DSPEC, wts)
    ref = oracle.net_maps(frames[0], DSPEC, wts)
    assert np.max(np.abs(maps - ref)) <= 1e-12 * (1 + np.max(np.abs(ref)))


def test_loss_and_gradients_match_torch_autograd():
    frames, truths = data()
    wts = weights()
    assert len(truths[0]) >= 2
    L, G = T.batch_grads(frames, truths, SPEC, wts)
    Lt, Gt = torch_loss(frames, truths, SPEC, wts)
    assert abs(L["total"] - Lt) <= 1e-10 * abs(Lt)
    for k in G:
        ref = Gt[k]
        err = np.linalg.norm(G[k] - ref) / (np.linalg.norm(ref) + 1e-300)
        assert err <= 1e-9, (k, err)


def test_finite_differences():
    frames, truths = data(n=1, empty_last=False)
    wts = weights(4)
    _, G = T.batch_grads(frames, truths, SPEC, wts)
    r = np.random.default_rng(7)
    for name in ["stem.w", "blk0.w1", "blk1.w2", "blk1.b1", "head.w", "head.b"]:
        for _ in range(2):
            idx = tuple(int(r.integers(0, s)) for s in wts[name].shape)
            h = 1e-5
            wp = {k: np.asarray(v, np.float64).copy() for k, v in wts.items()}
            wm = {k: np.asarray(v, np.float64).copy() for k, v in wts.items()}
            wp[name][idx] += h
            wm[name][idx] -= h
            Lp, _ = T.batch_grads(frames, truths, SPEC, wp)
            Lm, _ = T.batch_grads(frames, truths, SPEC, wm)
            fd = (Lp["total"] - Lm["total"]) / (2 * h)
            assert abs(fd - G[name][idx]) <= 1e-5 * (abs(fd) + 1e-3), (name, idx, fd, G[name][idx])


def test_count_term_closed_form():
    h, w = 6, 7
    maps = np.zeros((10, h, w))
    truth = np.zeros(3, S.TRUTH_DTYPE)
    truth["x"], truth["y"] = [0.5, 3.2, 6.9], [0.5, 2.2, 5.1]
    L, _ = T.frame_loss(maps, truth, SPEC)
    P = h * w
    v = P / 4 + T.VAR_EPS
    assert abs(L["count"] - (0.5 * math.log(2 * math.pi * v) + (3 - P / 2) ** 2 / (2 * v))) <= 1e-12
    # BCE at logit 0: log 2 everywhere
    assert abs(L["bce"] - math.log(2.0)) <= 1e-12


def test_localisation_term_with_one_dominant_pixel():
    h, w = 5, 6
    maps = np.zeros((10, h, w))
    maps[0] = -40.0
    maps[0, 2, 3] = 40.0
    maps[1, 2, 3], maps[2, 2, 3], maps[3, 2, 3], maps[4, 2, 3] = 0.1, -0.2, 0.3, 2.0
    maps[5:9, 2, 3] = [0.2, -0.1, 0.5, 1.0]
    truth = np.zeros(1, S.TRUTH_DTYPE)
    truth["x"], truth["y"], truth["z_nm"], truth["photons"] = 3.7, 2.1, 140.0, 2500.0
    L, _ = T.frame_loss(maps, truth, SPEC)
    t = [3.7, 2.1, 140.0 / SPEC.z_scale, 2500.0 / SPEC.ph_scale]
    m = [3 + 0.5 + 0.1, 2 + 0.5 - 0.2, 0.3, 2.0]
    s = oracle.softplus(np.array([0.2, -0.1, 0.5, 1.0])) + 0.01
    nll = sum(0.5 * math.log(2 * math.pi) + math.log(s[d]) + (t[d] - m[d]) ** 2 / (2 * s[d] ** 2) for d in range(4))
    assert abs(L["loc"] - nll) <= 1e-9


def test_transposed_conv_is_the_adjoint():
    r = np.random.default_rng(9)
    for d in (1, 3):
        x = r.standard_normal((5, 11, 13))
        y = r.standard_normal((4, 11, 13))
        W = r.standard_normal((4, 5, 3, 3))
        lhs = np.sum(oracle.conv3x3(x, W, None, d) * y)
        rhs = np.sum(x * oracle.conv3x3(y, T._flip_t(W), None, d))
        assert abs(lhs - rhs) <= 1e-10 * abs(lhs)
        # the weight gradient is the derivative of <conv(x), y> with respect to W
        g = T._wgrad(y, x, d)
        k = (1, 2, 0, 2)
        Wp = W.copy()
        Wp[k] += 1.0
        assert abs(np.sum(oracle.conv3x3(x, Wp, None, d) * y) - lhs - g[k]) <= 1e-9 * (1 + abs(g[k]))
