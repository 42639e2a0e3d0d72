"""Pins of the predictor's CPU reference (CPU only): convolution against
scipy's correlation, the FP64 backward against central finite differences,
bfloat16 rounding, the weighted BCE and Adam against torch's CPU routines."""
import numpy as np
import pytest
import scipy.signal
import torch

from oracle import cnn

RNG = np.random.default_rng(7)


@pytest.mark.parametrize("d", [2, 3])
def test_conv_matches_scipy(d):
    n = 6 if d == 3 else 9
    x = RNG.normal(size=(2, 3) + (n,) * d)
    w = RNG.normal(size=(4, 3) + (3,) * d)
    b = RNG.normal(size=4)
    y = cnn.conv_valid(x, w, b)
    for i in range(2):
        for o in range(4):
            ref = sum(scipy.signal.correlate(x[i, c], w[o, c], mode="valid") for c in range(3)) + b[o]
            assert np.allclose(y[i, o], ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("d", [2, 3])
def test_backward_finite_differences(d):
    n = 4 if d == 3 else 5
    c0, c1 = 3, 4
    x = RNG.normal(size=(2, c0) + (n + 6,) * d)
    y = (RNG.random(size=(2,) + (n,) * d) < 0.3).astype(float)
    params = cnn.init_params(c0, c1, d, seed=3)
    params = [p + 0.01 * RNG.normal(size=np.shape(p)) for p in params]
    loss, grads = cnn.backward(x, params, y, pos_weight=3.0)
    h = 1e-6
    for pi in range(6):
        flat = params[pi].ravel()
        idxs = RNG.choice(flat.size, size=min(6, flat.size), replace=False)
        for i in idxs:
            pp = [p.copy() for p in params]
            pm = [p.copy() for p in params]
            pp[pi].ravel()[i] += h
            pm[pi].ravel()[i] -= h
            lp = cnn.bce_with_logits(cnn.forward(x, pp)[0], y, 3.0)[0]
            lm = cnn.bce_with_logits(cnn.forward(x, pm)[0], y, 3.0)[0]
            fd = (lp - lm) / (2 * h)
            g = grads[pi].ravel()[i]
            assert abs(fd - g) <= 1e-6 * max(1.0, abs(g)) + 1e-9, (pi, i, fd, g)


def test_bf16_round_matches_torch():
    x = np.concatenate([RNG.normal(size=1000).astype(np.float32),
                        np.array([1.0, -0.0, 3.0e38, 1e-40, 1.00390625, 1.01171875], np.float32)])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(cnn.bf16_round(x), ref)


def test_bce_matches_torch():
    z = RNG.normal(size=(3, 8, 8)) * 4
    y = (RNG.random(size=(3, 8, 8)) < 0.2).astype(float)
    loss, grad = cnn.bce_with_logits(z, y, 5.0)
    zt = torch.tensor(z, requires_grad=True)
    lt = torch.nn.functional.binary_cross_entropy_with_logits(
        zt, torch.tensor(y), pos_weight=torch.tensor(5.0))
    lt.backward()
    assert loss == pytest.approx(lt.item(), rel=1e-12)
    assert np.allclose(grad, zt.grad.numpy(), rtol=1e-10, atol=1e-14)


def test_adam_matches_torch():
    p = [RNG.normal(size=(4, 3)).astype(np.float32)]
    g = [RNG.normal(size=(4, 3)).astype(np.float32)]
    m = [np.zeros((4, 3), np.float32)]
    v = [np.zeros((4, 3), np.float32)]
    pt = torch.tensor(p[0], requires_grad=True)
    opt = torch.optim.Adam([pt], lr=1e-2)
    for t in range(1, 4):
        p, m, v = cnn.adam_step(p, g, m, v, t, 1e-2)
        pt.grad = torch.tensor(g[0])
        opt.step()
    assert np.allclose(p[0], pt.detach().numpy(), rtol=1e-6, atol=1e-7)
