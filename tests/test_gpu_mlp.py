"""GPU kernels of the precision-proposal network against the float64
reference (oracle/mlp.py): forward, loss, backward, Adam, and a short
training run.

Tolerances come from float32 accumulation: a length-n dot product carries at
most n * 2^-24 times the sum of |terms| of rounding error, so every output
is compared against the same network evaluated on |W| and |x| (the size of
the terms), scaled by a bound of 4 layers x 67 terms x 2^-24 < 2e-5.  Samples
whose float64 pre-activations come within 1e-3 of zero are left out, so both
sides take the same ReLU branch."""
import numpy as np
import pytest

from oracle import mlp
from tests.gpu_util import log

pytestmark = pytest.mark.gpu

EPS32 = 2.0 ** -24
BOUND = 4 * 67 * EPS32


def _pre_activations(theta, X):
    p = mlp.unpack(theta)
    z1 = X @ p["W1"].T + p["b1"]
    z2 = np.maximum(z1, 0) @ p["W2"].T + p["b2"]
    z3 = np.maximum(z2, 0) @ p["W3"].T + p["b3"]
    return z1, z2, z3


def _case(seed, batch):
    rng = np.random.default_rng(seed)
    theta = mlp.init(seed)
    # small random biases so both ReLU branches occur
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in mlp.SHAPES])
    for k, (name, _) in enumerate(mlp.SHAPES):
        if name.startswith("b"):
            theta[offs[k]:offs[k + 1]] = rng.normal(scale=0.1, size=offs[k + 1] - offs[k])
    theta = theta.astype(np.float32).astype(np.float64)   # exactly representable in fp32
    X = rng.uniform(-1.5, 1.5, size=(4 * batch, mlp.NI)).astype(np.float32).astype(np.float64)
    z1, z2, z3 = _pre_activations(theta, X)
    keep = np.min(np.abs(np.concatenate([z1, z2, z3], 1)), 1) > 1e-3
    X = X[keep][:batch]
    assert len(X) == batch
    return theta, X


def _dev(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float32).reshape(-1), device="cuda")


@pytest.mark.parametrize("seed,batch", [(0, 1), (1, 37), (2, 300)])
def test_forward_and_backward_match_reference(hk, seed, batch):
    import torch
    log("mlp fwd/bwd seed=%d batch=%d" % (seed, batch))
    theta, X = _case(seed, batch)
    rng = np.random.default_rng(50 + seed)
    T = rng.normal(size=(batch, 2)).astype(np.float32).astype(np.float64)
    W = _dev(theta)
    Xd = _dev(X).view(batch, 3)
    cache = torch.empty(batch * hk.mlp_cache_floats(), dtype=torch.float32, device="cuda")
    Y = hk.mlp_forward(W, Xd, cache)
    loss, dY = hk.mlp_mse(Y, _dev(T).view(batch, 2))
    dW = hk.mlp_backward(W, cache, dY)
    torch.cuda.synchronize()
    # reference, and the same network on |W|, |x| for the size of the terms
    Yr, acts = mlp.forward(theta, X)
    Ya, abs_acts = mlp.forward(np.abs(theta), np.abs(X))
    Yg = Y.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(Yg - Yr) <= BOUND * Ya + 1e-30)
    # the cache holds the input and the hidden activations
    cg = cache.cpu().numpy().reshape(batch, -1).astype(np.float64)
    assert np.all(np.abs(cg - np.concatenate(acts, 1)) <= BOUND * np.concatenate(abs_acts, 1) + 1e-30)
    # loss and dY from the GPU outputs
    Lr, dYr = mlp.mse(Yg, T)
    assert abs(loss.item() - Lr) <= 8 * EPS32 * (Lr + 1e-30) * 2 * batch
    np.testing.assert_allclose(dY.cpu().numpy(), dYr, rtol=4 * EPS32, atol=1e-30)
    # gradient of sum(dY * Y): the reference with the same dY
    dYg = dY.cpu().numpy().astype(np.float64)
    gr = mlp.backward(theta, acts, dYg)
    ga = mlp.backward(np.abs(theta), abs_acts, np.abs(dYg))
    gg = dW.cpu().numpy().astype(np.float64)
    tol = (BOUND + batch * EPS32) * ga + 1e-30
    bad = np.abs(gg - gr) > tol
    assert not bad.any(), (np.nonzero(bad)[0][:10], gg[bad][:5], gr[bad][:5])


def test_backward_is_reproducible(hk):
    import torch
    theta, X = _case(5, 200)
    W, Xd = _dev(theta), _dev(X).view(200, 3)
    cache = torch.empty(200 * hk.mlp_cache_floats(), dtype=torch.float32, device="cuda")
    Y = hk.mlp_forward(W, Xd, cache)
    dY = torch.ones_like(Y)
    g1 = hk.mlp_backward(W, cache, dY)
    g2 = hk.mlp_backward(W, cache, dY)
    assert torch.equal(g1, g2)


def test_adam_step_matches_reference(hk):
    import torch
    rng = np.random.default_rng(9)
    n = hk.mlp_nparams()
    theta = rng.normal(size=n).astype(np.float32).astype(np.float64)
    m = np.zeros(n)
    v = np.zeros(n)
    W, md, vd = _dev(theta), torch.zeros(n, device="cuda"), torch.zeros(n, device="cuda")
    # the kernel takes float32 hyper-parameters: give the reference the same values
    f32 = lambda x: float(np.float32(x))
    lr, b1, b2, eps = f32(1e-2), f32(0.9), f32(0.999), f32(1e-8)
    for step in range(1, 6):
        g = rng.normal(size=n).astype(np.float32).astype(np.float64)
        theta, m, v = mlp.adam_step(theta, m, v, g, step, lr=lr, b1=b1, b2=b2, eps=eps)
        hk.mlp_adam_step(W, md, vd, _dev(g), step, lr, b1, b2, eps)
        torch.cuda.synchronize()
        np.testing.assert_allclose(md.cpu().numpy(), m, rtol=1e-5, atol=1e-7)
        np.testing.assert_allclose(vd.cpu().numpy(), v, rtol=1e-5, atol=1e-9)
        np.testing.assert_allclose(W.cpu().numpy(), theta, rtol=1e-5, atol=1e-5)


def test_gpu_training_reduces_loss_like_reference(hk):
    """Same data, same initial weights, full-batch Adam: the GPU loop of
    forward / loss / backward / Adam kernels starts at the reference's loss
    and ends within 50% of the reference's final loss (float32 and float64
    trajectories separate slowly over 300 steps)."""
    import torch
    rng = np.random.default_rng(7)
    X = rng.uniform(-1, 1, size=(128, 3))
    T = np.stack([np.sin(X[:, 0]) + X[:, 1] * X[:, 2], X[:, 0] - 0.5 * X[:, 1] ** 2], 1)
    theta0 = mlp.init(7).astype(np.float32).astype(np.float64)
    X = X.astype(np.float32).astype(np.float64)
    T = T.astype(np.float32).astype(np.float64)
    _, hist = mlp.train(theta0, X, T, steps=300, lr=3e-3)
    W = _dev(theta0)
    m = torch.zeros_like(W)
    v = torch.zeros_like(W)
    Xd, Td = _dev(X).view(128, 3), _dev(T).view(128, 2)
    cache = torch.empty(128 * hk.mlp_cache_floats(), dtype=torch.float32, device="cuda")
    losses = []
    for step in range(1, 301):
        Y = hk.mlp_forward(W, Xd, cache)
        loss, dY = hk.mlp_mse(Y, Td)
        losses.append(loss)
        hk.mlp_adam_step(W, m, v, hk.mlp_backward(W, cache, dY), step, 3e-3)
    lg = [x.item() for x in losses]
    log("loss ref %.4g -> %.4g, gpu %.4g -> %.4g" % (hist[0], hist[-1], lg[0], lg[-1]))
    assert abs(lg[0] - hist[0]) <= 1e-5 * hist[0]
    assert lg[-1] < 0.05 * lg[0]
    assert abs(lg[-1] - hist[-1]) <= 0.5 * hist[-1]
