"""Pins of the U-Net oracle against library routines, adjoint identities, finite
differences and closed forms (no GPU)."""
import numpy as np
import pytest
import torch
from scipy.signal import correlate2d

from oracle import unet as U


def test_bf16_rounding_matches_torch_and_ties_to_even():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(5000) * 10.0 ** rng.integers(-6, 6, 5000),
                        [0.0, -0.0, 1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -(1 + 2 ** -8), 65504.0]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(U.to_bf16(x), ref)
    # halfway cases go to the even mantissa
    assert U.to_bf16(np.array([1 + 2 ** -8]))[0] == 1.0
    assert U.to_bf16(np.array([1 + 3 * 2 ** -8]))[0] == 1 + 2 ** -6


def test_param_count_closed_form():
    a = U.Arch(levels=4, base=32)
    C = [32, 64, 128, 256]
    n = 0
    n += 32 * 9 * 1 + 32 + 32 * 9 * 32 + 32
    for l in range(1, 4):
        n += C[l] * 9 * C[l - 1] + C[l] + C[l] * 9 * C[l] + C[l]
    for l in range(2, -1, -1):
        n += C[l] * 9 * (C[l + 1] + C[l]) + C[l] + C[l] * 9 * C[l] + C[l]
    n += 32 + 1
    assert a.n_params() == n
    theta = U.init_params(a, 0)
    assert theta.size == n
    assert np.array_equal(U.pack(a, U.unpack(a, theta)), theta)


def test_conv3x3_equals_scipy_correlate():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 7, 9, 3))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    y = U.conv3x3(x, w, b)
    for n in range(2):
        for o in range(4):
            ref = b[o] + sum(correlate2d(x[n, :, :, c], w[o, :, :, c], mode="same") for c in range(3))
            assert np.allclose(y[n, :, :, o], ref, atol=1e-12)


def test_conv_gradients_are_adjoints():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, 6, 8, 3))
    w = rng.standard_normal((5, 3, 3, 3))
    dy = rng.standard_normal((2, 6, 8, 5))
    lhs = float(np.sum(U.conv3x3(x, w, None) * dy))
    assert np.isclose(lhs, float(np.sum(x * U.conv3x3_dgrad(dy, w))), rtol=1e-12)
    dw, db = U.conv3x3_wgrad(dy, x)
    assert np.isclose(lhs, float(np.sum(w * dw)), rtol=1e-12)
    assert np.allclose(db, dy.sum(axis=(0, 1, 2)))


def test_pool_and_upsample_adjoints():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, 8, 6, 3))
    y = rng.standard_normal((2, 4, 3, 3))
    assert np.isclose(np.sum(U.avgpool2(x) * y), np.sum(x * U.avgpool2_back(y)), rtol=1e-12)
    assert np.isclose(np.sum(U.up2(y) * x), np.sum(y * U.up2_back(x)), rtol=1e-12)
    assert np.allclose(U.avgpool2(np.ones((1, 4, 4, 1))), 1.0)


@pytest.mark.parametrize("levels", [1, 2, 3])
def test_network_gradient_matches_finite_differences(levels):
    arch = U.Arch(levels=levels, base=2)
    rng = np.random.default_rng(10 + levels)
    theta = U.init_params(arch, 4) + 0.05 * rng.standard_normal(arch.n_params())
    h, w = 8, 12
    fbp = rng.standard_normal((2, h, w))
    target = fbp + 0.3 * rng.standard_normal((2, h, w))
    s = 1.7
    loss, g = U.loss_and_grad(arch, theta, fbp, target, s)
    idx = rng.choice(arch.n_params(), 25, replace=False)
    eps = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += eps
        tm[i] -= eps
        fd = (U.loss_and_grad(arch, tp, fbp, target, s)[0] - U.loss_and_grad(arch, tm, fbp, target, s)[0]) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * (abs(fd) + 1e-3), (i, fd, g[i])
    # the loss is the mean squared error of x0 against the target, scaled by 1/s^2
    x0, _, _ = U.forward(arch, theta, fbp, s)
    assert np.isclose(loss, np.mean((x0 - target) ** 2) / s ** 2, rtol=1e-12)


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(5)
    th = rng.standard_normal(50)
    g = rng.standard_normal(50)
    new, m, v = U.adam_step(th, g, np.zeros(50), np.zeros(50), 1, lr=1e-2)
    assert np.allclose(new, th - 1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_oracle_training_reduces_loss():
    arch = U.Arch(levels=2, base=2)
    rng = np.random.default_rng(6)
    theta = U.init_params(arch, 1)
    fbp = rng.standard_normal((3, 8, 8))
    target = fbp + 0.5 * U.avgpool2_back(U.avgpool2(fbp[..., None]))[..., 0]
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    l0 = U.loss_and_grad(arch, theta, fbp, target, 1.0)[0]
    for k in range(1, 61):
        loss, g = U.loss_and_grad(arch, theta, fbp, target, 1.0)
        theta, m, v = U.adam_step(theta, g, m, v, k, lr=3e-3)
    assert loss < 0.5 * l0
