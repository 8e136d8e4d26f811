"""GPU parity of the U-Net kernels and network against the FP64 oracle (oracle/unet.py).

Tolerances.  A matrix-core convolution takes bfloat16 operands exactly and accumulates in
float32, then rounds to bfloat16 (unit roundoff u = 2^-9); the oracle evaluates the same
bfloat16 operands in float64 and rounds the same way.  The float32 accumulation error
(< K 2^-24 relative, K <= 3456) is far below u, so single layers agree to one bfloat16 ulp
(at most 2^-7 relative) where a value sits near a rounding boundary and exactly elsewhere.  Weight
gradients are float32 sums of exact products: relative L2 <= 1e-5.  Through the whole
network the occasional one-ulp differences propagate: with ~15 rounding stages the output
residual r agrees to relative L2 <= 1e-2 (measured ~1e-3) and parameter gradients to <= 3e-2
per layer; the loss to 1e-3.  The Adam update is float32 arithmetic on the GPU's own
gradient: 1e-6.
"""
import numpy as np
import pytest
import torch

from oracle import unet as U

from gpu_util import dev

pytestmark = pytest.mark.gpu


def _bf(a) -> torch.Tensor:
    return torch.as_tensor(np.asarray(a, dtype=np.float32)).to(torch.bfloat16).to(dev())


def _np(t: torch.Tensor) -> np.ndarray:
    torch.cuda.synchronize()
    return t.detach().float().cpu().numpy().astype(np.float64)


def _ulp_close(got, ref, frac_max=0.02):
    # one bfloat16 ulp is 2^-8 .. 2^-7 of the value (7 stored mantissa bits)
    got, ref = np.asarray(got), np.asarray(ref)
    err = np.abs(got - ref)
    bound = 2.0 ** -7 * np.abs(ref) + 1e-30
    assert np.all(err <= bound * 1.0001 + 1e-6 * np.max(np.abs(ref))), float(np.max(err / (np.abs(ref) + 1e-30)))
    assert np.mean(err > 0) <= frac_max


@pytest.mark.parametrize("cin,cout,W,off", [(32, 64, 70, 0), (64, 96, 33, 32), (96, 32, 130, 8)])
def test_conv3x3_forward_relu(cin, cout, W, off):
    from paper_2603_28756_amd import tomo
    rng = np.random.default_rng(cin + cout + W)
    B, H = 2, 5
    ld = cin + off + 8
    xb = rng.standard_normal((B, H, W, ld))
    x = _bf(xb)
    w = _bf(rng.standard_normal((cout, 3, 3, cin)) / np.sqrt(9 * cin))
    bias = torch.as_tensor(rng.standard_normal(cout), dtype=torch.float32, device=dev())
    out = torch.zeros((B, H, W, cout + 16), dtype=torch.bfloat16, device=dev())
    xin = x[..., off:]
    tomo.nn_conv3x3(xin, w, bias, cin, cout, relu=True, out=out, x_ld=ld, out_ld=cout + 16)
    xs = _np(x)[..., off:off + cin]
    ref = U.to_bf16(U.relu(U.conv3x3(xs, _np(w), _np(bias))))
    got = _np(out)
    _ulp_close(got[..., :cout], ref)
    assert np.all(got[..., cout:] == 0.0)  # untouched channels beyond cout


@pytest.mark.parametrize("co", [32, 96])
def test_conv3x3_masked_input_gradient_form(co):
    from paper_2603_28756_amd import tomo
    rng = np.random.default_rng(9)
    B, H, W, ci = 3, 7, 40, 64
    dz = _bf(rng.standard_normal((B, H, W, ci)))
    w = _bf(rng.standard_normal((co, 3, 3, ci)) / 20)
    mask = _bf(rng.standard_normal((B, H, W, co)))
    out = tomo.nn_conv3x3(dz, w, None, ci, co, mask=mask)
    ref = U.to_bf16(U.conv3x3(_np(dz), _np(w), None) * (_np(mask) > 0))
    _ulp_close(_np(out), ref)


# widths that are multiples of 32 take the haloed row-tile kernel: one-row images (both halo
# rows outside), 32-pixel rows (both halo columns outside, chunks crossing slices) and several
# channel tiles on both sides; the other widths take the per-tap kernel
@pytest.mark.parametrize("B,H,W,cin,cout", [(2, 5, 70, 32, 64), (2, 64, 96, 64, 32), (1, 9, 17, 96, 96),
                                            (3, 1, 32, 96, 64), (2, 7, 64, 32, 96), (1, 40, 128, 64, 64)])
def test_conv3x3_weight_gradient(B, H, W, cin, cout):
    from paper_2603_28756_amd import tomo
    rng = np.random.default_rng(B * H + W)
    dz = _bf(rng.standard_normal((B, H, W, cout)))
    x = _bf(rng.standard_normal((B, H, W, cin)))
    dw, db = tomo.nn_conv3x3_wgrad(dz, x, cin, cout)
    rw, rb = U.conv3x3_wgrad(_np(dz), _np(x))
    assert np.linalg.norm(_np(dw) - rw) / np.linalg.norm(rw) < 1e-5
    assert np.linalg.norm(_np(db) - rb) / np.linalg.norm(rb) < 1e-5


def _net_case(levels=3, H=48, W=40, B=2, seed=0, base=32):
    arch = U.Arch(levels=levels, base=base)
    rng = np.random.default_rng(seed)
    theta = U.init_params(arch, seed) + 0.01 * rng.standard_normal(arch.n_params())
    theta = theta.astype(np.float32).astype(np.float64)
    yy, xx = np.mgrid[0:H, 0:W]
    fbp = np.stack([np.sin(0.3 * yy + 0.2 * k) * np.cos(0.25 * xx) + 0.3 * rng.standard_normal((H, W))
                    for k in range(B)]).astype(np.float32).astype(np.float64)
    target = (fbp + 0.2 * rng.standard_normal(fbp.shape)).astype(np.float32).astype(np.float64)
    return arch, theta, fbp, target


# 64 base channels: the 64-channel forms of the first layer and of the head-writing last
# convolution
@pytest.mark.parametrize("levels,H,W,base", [(3, 48, 40, 32), (4, 64, 72, 32), (1, 16, 24, 32),
                                             (2, 40, 56, 64)])
def test_network_forward(levels, H, W, base):
    from paper_2603_28756_amd import tomo
    arch, theta, fbp, _ = _net_case(levels, H, W, base=base)
    s = 1.3
    net = tomo.UNet(H, W, levels=levels, base=base, max_batch=3)
    assert net.n_params == arch.n_params()
    net.set_params(torch.as_tensor(theta, dtype=torch.float32))
    x0 = net.forward(torch.as_tensor(fbp, dtype=torch.float32, device=dev()).contiguous(), s)
    r_gpu = (_np(x0) - fbp) / s
    _, r_ref, _ = U.forward(arch, theta, fbp, s, bf16=True)
    assert np.linalg.norm(r_gpu - r_ref) / np.linalg.norm(r_ref) < 1e-2
    _, r_exact, _ = U.forward(arch, theta, fbp, s, bf16=False)
    assert np.linalg.norm(r_gpu - r_exact) / np.linalg.norm(r_exact) < 5e-2


# (levels, H, W, base channels, max_batch, batch).  128 x 128 at batch 5 of 8 needs more
# weight-gradient split scratch than the full batch (the split count is not monotone in the
# pixel count); 96 base channels give 12 first-layer channel groups (not a power of two).
@pytest.mark.parametrize("levels,H,W,base,max_batch,B", [
    (3, 48, 40, 32, 2, 2), (2, 32, 96, 32, 2, 2), (2, 128, 128, 32, 8, 5), (2, 32, 64, 96, 2, 2)])
def test_network_loss_and_gradient(levels, H, W, base, max_batch, B):
    from paper_2603_28756_amd import tomo
    arch, theta, fbp, target = _net_case(levels, H, W, B=B, seed=levels, base=base)
    s = 0.9
    net = tomo.UNet(H, W, levels=levels, base=base, max_batch=max_batch)
    net.set_params(torch.as_tensor(theta, dtype=torch.float32))
    loss, g = net.loss_grad(torch.as_tensor(fbp, dtype=torch.float32, device=dev()).contiguous(),
                            torch.as_tensor(target, dtype=torch.float32, device=dev()).contiguous(), s)
    rl, rg = U.loss_and_grad(arch, theta, fbp, target, s, bf16=True)
    assert abs(loss - rl) / rl < 1e-3
    g = _np(g)
    gp, rp = U.unpack(arch, g), U.unpack(arch, rg)
    for name in gp:
        for a, b in zip(gp[name], rp[name]):
            a, b = np.ravel(a), np.ravel(b)
            assert np.linalg.norm(a - b) / (np.linalg.norm(b) + 1e-30) < 3e-2, name


def test_adam_step_and_training_reduces_loss():
    from paper_2603_28756_amd import tomo
    arch, theta, fbp, target = _net_case(2, 32, 32, B=2, seed=5)
    s, lr = 1.0, 1e-3
    net = tomo.UNet(32, 32, levels=2, base=32, max_batch=2)
    net.set_params(torch.as_tensor(theta, dtype=torch.float32))
    f = torch.as_tensor(fbp, dtype=torch.float32, device=dev()).contiguous()
    t = torch.as_tensor(target, dtype=torch.float32, device=dev()).contiguous()
    l0, g = net.loss_grad(f, t, s)
    th0 = _np(net.params())
    net.train_step(f, t, s, lr)
    th1 = _np(net.params())
    ref, _, _ = U.adam_step(th0, _np(g), np.zeros_like(th0), np.zeros_like(th0), 1, lr)
    assert np.max(np.abs(th1 - ref)) <= 1e-6 * max(1.0, np.max(np.abs(ref)))
    for _ in range(60):
        net.train_step(f, t, s, lr)
    l1, _ = net.loss_grad(f, t, s)
    assert l1 < 0.7 * l0
