"""Surrogate network kernels (forward, backward, Adam) against the FP64 MLP
oracle, through the C ABI, on seeded parameters and batches."""
import numpy as np
import pytest

import synth
from oracle import mlp as omlp

pytestmark = pytest.mark.gpu


def _params(seed=3):
    theta = synth.mlp_init(918).astype(np.float64)
    theta += 0.05 * np.random.default_rng(seed).standard_normal(theta.size)
    return theta.astype(np.float32)


@pytest.mark.parametrize("B", [1, 16, 37, 256, 1000])
def test_forward_and_gradient_match_the_fp64_oracle(gpu_available, B):
    import torch
    from paper_1601_00918_amd import mlp
    p32 = _params()
    X, t = synth.mlp_batch(B, seed=B)
    net = mlp.Network(p32, max_batch=B)
    Xd, td = torch.from_numpy(X).cuda(), torch.from_numpy(t).cuda()
    loss, grad = net.gradient(Xd, td)
    torch.cuda.synchronize()
    y_gpu = net.y[:B].cpu().numpy().astype(np.float64)
    g_gpu = grad.cpu().numpy().astype(np.float64)
    theta = p32.astype(np.float64)
    y_ref, _ = omlp.forward(theta, X.astype(np.float64))
    L_ref, g_ref = omlp.backward(theta, X.astype(np.float64), t.astype(np.float64))
    ey = np.abs(y_gpu - y_ref).max() / np.abs(y_ref).max()
    # per parameter block: max |dg| / max |g|
    eg = []
    for (gw, gb), (rw, rb) in zip(omlp.unpack(g_gpu), omlp.unpack(g_ref)):
        for a, b in ((gw, rw), (gb, rb)):
            eg.append(np.abs(a - b).max() / max(np.abs(b).max(), 1e-30))
    el = abs(float(loss.cpu()) / L_ref - 1)
    print("B=%d  y %.2e  grad blocks %s  loss %.2e" % (B, ey, ["%.1e" % e for e in eg], el),
          flush=True)
    assert ey <= 1e-5
    assert max(eg) <= 1e-4
    assert el <= 1e-5


def test_adam_matches_the_oracle_step(gpu_available):
    import torch
    from paper_1601_00918_amd import mlp
    rng = np.random.default_rng(11)
    p = _params()
    g = rng.standard_normal(p.size).astype(np.float32)
    m = (0.1 * rng.standard_normal(p.size)).astype(np.float32)
    v = (0.01 * rng.random(p.size)).astype(np.float32)
    P, G, M, V = (torch.from_numpy(a.copy()).cuda() for a in (p, g, m, v))
    mlp.adam(P, G, M, V, 7, lr=2e-3, beta1=0.9, beta2=0.999, eps=1e-8)
    # the kernel receives the hyperparameters as float32: give the oracle the
    # same values
    f32 = lambda a: float(np.float32(a))  # noqa: E731
    b1, b2, lr = f32(0.9), f32(0.999), f32(2e-3)
    ref, rm, rv = omlp.adam_step(p.astype(np.float64), g.astype(np.float64),
                                 m.astype(np.float64), v.astype(np.float64), 7, lr=lr,
                                 beta1=b1, beta2=b2, eps=f32(1e-8))
    # FP32 rounding of each update: a few units in the last place of its
    # operands (the moments cancel, so the bound is on the operands, not on
    # the result)
    u = 2.0 ** -24
    m64, v64, g64 = m.astype(np.float64), v.astype(np.float64), g.astype(np.float64)
    assert np.all(np.abs(M.cpu().numpy() - rm) <= 4 * u * (b1 * np.abs(m64) + (1 - b1) * np.abs(g64)))
    assert np.all(np.abs(V.cpu().numpy() - rv) <= 4 * u * (b2 * v64 + (1 - b2) * g64 * g64))
    # the step lr * mhat / (sqrt(vhat) + eps) carries the moments' errors
    c1, c2 = 1 - b1 ** 7, 1 - b2 ** 7
    den = np.sqrt(rv / c2) + 1e-8
    dm = 4 * u * (b1 * np.abs(m64) + (1 - b1) * np.abs(g64)) / c1
    bound = lr * (dm / den + 8 * u * np.abs(rm / c1) / den) + 2 * u * np.abs(ref)
    assert np.all(np.abs(P.cpu().numpy() - ref) <= bound + 1e-12)


def test_training_follows_the_oracle_and_reduces_the_loss(gpu_available):
    """Ten Adam steps on the same minibatches: the GPU loss trajectory stays
    within 1e-3 of the FP64 one and the loss of a smooth target falls.
    Adam divides each gradient by its own magnitude, so a parameter whose
    gradient is at the FP32 rounding level may step by lr in either
    direction: parameters are compared by the fraction that agree to 1e-5,
    not by their maximum difference."""
    import torch
    from paper_1601_00918_amd import mlp
    rng = np.random.default_rng(5)
    X = rng.uniform(-1, 1, (512, 6)).astype(np.float32)
    t = (np.sin(2 * X[:, 0]) + X[:, 1] * X[:, 2] - 0.5 * X[:, 3] ** 2).astype(np.float32)
    p0 = synth.mlp_init(918)
    net = mlp.Network(p0, max_batch=128)
    theta = p0.astype(np.float64)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    losses, ref_losses = [], []
    for k in range(1, 11):
        idx = rng.choice(512, 128, replace=False)
        xb, tb = X[idx], t[idx]
        loss = net.train_step(torch.from_numpy(xb).cuda(), torch.from_numpy(tb).cuda(), lr=3e-3)
        losses.append(float(loss.cpu()))
        L, g = omlp.backward(theta, xb.astype(np.float64), tb.astype(np.float64))
        ref_losses.append(L)
        theta, m, v = omlp.adam_step(theta, g, m, v, k, lr=3e-3)
    got = net.params.cpu().numpy().astype(np.float64)
    agree = float(np.mean(np.abs(got - theta) <= 1e-5))
    rel = max(abs(a / b - 1) for a, b in zip(losses, ref_losses))
    print("loss rel diff %.2e  params agreeing to 1e-5: %.4f  losses %s" % (
        rel, agree, ["%.3f" % l for l in losses]), flush=True)
    assert rel <= 1e-3
    assert agree >= 0.99
    assert losses[-1] < 0.7 * losses[0]
