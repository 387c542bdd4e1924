"""GPU parity of the tile-gate kernels (pooling, forward, backward, BCE, Adam)
against the FP64 oracle.  Bars: forward logits within 1e-5 relative; gradients
within 1e-4 per-tensor L2-relative; reproducible bit for bit."""
import numpy as np
import pytest

import oracle
import smlm_synth as S

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no HIP device", allow_module_level=True)
import paper_2410_02314_amd as dl  # noqa: E402

DEV = torch.device("cuda:0")
SEGMENTS = [("W1", 0, 72), ("b1", 72, 80), ("W2", 80, 656), ("b2", 656, 664), ("fw", 664, 672), ("fb", 672, 673)]


def theta_for(seed):
    th = S.gate_flat(S.gate_init(seed)).astype(np.float64)
    r = np.random.default_rng(seed + 1)
    th[72:80] = r.standard_normal(8) * 0.2
    th[656:664] = r.standard_normal(8) * 0.2
    th[672] = 0.3
    return th


def pooled_inputs(n, seed):
    """Seeded pooled tiles with the statistics of preprocessed frames
    (background about 1, bright blobs).  The values are FP32-representable,
    so the oracle and the kernels see the same input and pick the same
    maximising pixel of each channel (the global pool is a max)."""
    r = np.random.default_rng(seed)
    p = 1.0 + 0.1 * r.standard_normal((n, 64, 64))
    for b in range(n):
        for _ in range(r.integers(0, 6)):
            i, j = r.integers(0, 64, 2)
            p[b, max(0, i - 1):i + 2, max(0, j - 1):j + 2] += r.uniform(2, 10)
    return p.astype(np.float32).astype(np.float64)


def t32(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(DEV)


def test_gate_pool_matches_oracle():
    frames = S.render_frames(2, 512, 768, "sparse", 77)
    pooled = torch.empty((2 * 2 * 3, 64, 64), dtype=torch.float32, device=DEV)
    dl.gate_pool(torch.from_numpy(frames).to(DEV), pooled)
    torch.cuda.synchronize()
    g = pooled.cpu().numpy()
    k = 0
    for f in range(2):
        x = oracle.preprocess(frames[f], 0.5, 100.0, 0.01)
        for ty in range(2):
            for tx in range(3):
                ref = oracle.gate_pool(x[ty * 256:(ty + 1) * 256, tx * 256:(tx + 1) * 256], 4)
                assert np.max(np.abs(g[k] - ref)) <= 1e-6 * (1 + np.abs(ref).max())
                k += 1


def test_gate_forward_matches_oracle():
    p = pooled_inputs(37, 5)
    th = theta_for(3)
    logits = torch.empty(37, dtype=torch.float32, device=DEV)
    dl.gate_forward(t32(p), t32(th), logits)
    torch.cuda.synchronize()
    ref = oracle.gate_forward(p, th)
    got = logits.cpu().numpy()
    assert np.max(np.abs(got - ref) / (np.abs(ref) + 1e-3)) <= 1e-5


def test_gate_backward_matches_oracle_and_is_deterministic():
    n = 29
    p = pooled_inputs(n, 6)
    th = theta_for(4)
    dg = np.random.default_rng(8).standard_normal(n) / n
    work = torch.empty(n * 673, dtype=torch.float32, device=DEV)
    logits = torch.empty(n, dtype=torch.float32, device=DEV)
    grad = torch.empty(673, dtype=torch.float32, device=DEV)
    dl.gate_backward(t32(p), t32(th), t32(dg), work, logits, grad)
    torch.cuda.synchronize()
    got = grad.cpu().numpy().astype(np.float64)
    ref = oracle.gate_backward(p, th, dg)
    for name, a, b in SEGMENTS:
        rel = np.linalg.norm(got[a:b] - ref[a:b]) / max(np.linalg.norm(ref[a:b]), 1e-12)
        print(name, rel)
        assert rel <= 1e-4, name
    grad2 = torch.empty_like(grad)
    dl.gate_backward(t32(p), t32(th), t32(dg), work, logits, grad2)
    torch.cuda.synchronize()
    assert torch.equal(grad, grad2)


def test_gate_bce_and_adam_match_oracle():
    r = np.random.default_rng(9)
    g = r.standard_normal(300) * 4
    y = (r.random(300) < 0.4).astype(np.float64)
    loss = torch.empty(1, dtype=torch.float32, device=DEV)
    dlg = torch.empty(300, dtype=torch.float32, device=DEV)
    dl.gate_bce(t32(g), t32(y), loss, dlg)
    torch.cuda.synchronize()
    L, dref = oracle.bce(g.astype(np.float32).astype(np.float64), y)
    assert abs(loss.item() - L) <= 1e-6 * max(1, abs(L))
    assert np.max(np.abs(dlg.cpu().numpy() - dref)) <= 1e-7
    th = r.standard_normal(673)
    m = np.zeros(673)
    v = np.zeros(673)
    tg, mg, vg = t32(th), t32(m), t32(v)
    th_ref = th.astype(np.float32).astype(np.float64)
    for step in range(1, 4):
        grad = r.standard_normal(673)
        oracle.adam_step(th_ref, m, v, grad.astype(np.float32).astype(np.float64), step)
        dl.gate_adam(tg, mg, vg, t32(grad), step)
    torch.cuda.synchronize()
    assert np.max(np.abs(tg.cpu().numpy() - th_ref)) <= 1e-6
