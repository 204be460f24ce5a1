"""Pins of the FP64 denoiser oracle (CPU only).

Each layer is checked against an independent implementation (torch's CPU
conv3d / pooling / interpolation and autograd, torch.optim.Adam) or a closed
form, and the whole network's gradient against central finite differences,
so that a transposed tap, a swapped concatenation order or a dropped skip
path fails a test.
"""

import numpy as np
import pytest
import torch
import torch.nn.functional as F

from oracle import nn_oracle as nn


def _torch_w(w):
    co, _, ci = w.shape
    return torch.from_numpy(w.reshape(co, 3, 3, 3, ci).transpose(0, 4, 1, 2, 3).copy())


def _ncdhw(x):
    return torch.from_numpy(np.ascontiguousarray(x.transpose(0, 4, 1, 2, 3)))


def test_conv3d_matches_torch():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(2, 5, 6, 7, 3))
    w = rng.normal(size=(4, 27, 3))
    b = rng.normal(size=4)
    y = nn.conv3d(x, w, b)
    yt = F.conv3d(_ncdhw(x), _torch_w(w), torch.from_numpy(b), padding=1)
    np.testing.assert_allclose(y, yt.numpy().transpose(0, 2, 3, 4, 1), rtol=0, atol=1e-12)


def test_conv3d_tap_convention():
    """Tap t = 9(dz+1) + 3(dy+1) + (dx+1) reads the input at (z+dz, y+dy, x+dx)."""
    x = np.zeros((1, 5, 5, 5, 1))
    x[0, 2, 2, 2, 0] = 1.0
    for t, (dz, dy, dx) in enumerate(nn.TAPS):
        w = np.zeros((1, 27, 1))
        w[0, t, 0] = 1.0
        y = nn.conv3d(x, w, None)
        # y[v] = x[v + off]  -> the one nonzero output sits at (2,2,2) - off
        assert y[0, 2 - dz, 2 - dy, 2 - dx, 0] == 1.0 and y.sum() == 1.0


def test_conv3d_backward_matches_autograd():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(2, 4, 5, 6, 3))
    w = rng.normal(size=(5, 27, 3))
    dy = rng.normal(size=(2, 4, 5, 6, 5))
    dx, dw, db = nn.conv3d_backward(dy, x, w)
    xt = _ncdhw(x).requires_grad_(True)
    wt = _torch_w(w).requires_grad_(True)
    bt = torch.zeros(5, dtype=torch.float64, requires_grad=True)
    yt = F.conv3d(xt, wt, bt, padding=1)
    yt.backward(_ncdhw(dy))
    np.testing.assert_allclose(dx, xt.grad.numpy().transpose(0, 2, 3, 4, 1), atol=1e-11)
    dwt = wt.grad.numpy().transpose(0, 2, 3, 4, 1).reshape(5, 27, 3)
    np.testing.assert_allclose(dw, dwt, atol=1e-11)
    np.testing.assert_allclose(db, bt.grad.numpy(), atol=1e-11)


def test_pool_and_up_match_torch_and_are_adjoint():
    rng = np.random.default_rng(3)
    x = rng.normal(size=(2, 4, 6, 8, 3))
    p = nn.pool2(x)
    pt = F.avg_pool3d(_ncdhw(x), 2).numpy().transpose(0, 2, 3, 4, 1)
    np.testing.assert_allclose(p, pt, atol=1e-14)
    u = nn.up2(p)
    ut = F.interpolate(_ncdhw(p), scale_factor=2, mode="nearest").numpy().transpose(0, 2, 3, 4, 1)
    np.testing.assert_array_equal(u, ut)
    y = rng.normal(size=p.shape)
    assert abs((nn.pool2(x) * y).sum() - (x * nn.pool2_backward(y)).sum()) < 1e-12
    z = rng.normal(size=x.shape)
    assert abs((nn.up2(p) * z).sum() - (p * nn.up2_backward(z)).sum()) < 1e-12


def test_adam_matches_torch_optim():
    rng = np.random.default_rng(4)
    p = rng.normal(size=50)
    m = np.zeros(50)
    v = np.zeros(50)
    pt = torch.tensor(p.copy(), requires_grad=True)
    opt = torch.optim.Adam([pt], lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    for step in range(1, 6):
        g = rng.normal(size=50)
        p, m, v = nn.adam(p, g, m, v, step, 3e-3)
        pt.grad = torch.tensor(g)
        opt.step()
    np.testing.assert_allclose(p, pt.detach().numpy(), rtol=0, atol=1e-14)


def test_adam_first_step_is_lr_times_sign():
    g = np.array([1e-3, -2.0, 5.0])
    p, _, _ = nn.adam(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, 0.1, eps=0.0)
    np.testing.assert_allclose(p, -0.1 * np.sign(g), atol=1e-15)


def _random_params(levels, c0, cin, seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return {n: rng.normal(scale=scale, size=s) for n, s in nn.param_shapes(levels, c0, cin)}


def test_param_count_formula():
    # 4 levels of 16..128 channels, 16 input channels: 27 ci co + co per conv
    c = [16, 32, 64, 128]
    convs = [(16, 16), (16, 16), (16, 32), (32, 32), (32, 64), (64, 64), (64, 128), (128, 128),
             (64 + 128, 64), (64, 64), (32 + 64, 32), (32, 32), (16 + 32, 16), (16, 16)]
    n = sum(27 * ci * co + co for ci, co in convs) + c[0] + 1
    assert sum(int(np.prod(s)) for _, s in nn.param_shapes(4, 16, 16)) == n


@pytest.mark.parametrize("levels,c0,cin,shape", [(2, 2, 2, (1, 4, 4, 4)), (3, 2, 3, (2, 4, 4, 8))])
def test_unet_gradient_finite_differences(levels, c0, cin, shape):
    p = _random_params(levels, c0, cin, seed=5)
    rng = np.random.default_rng(6)
    x = rng.normal(size=shape + (cin,))
    tgt = rng.normal(size=shape)
    m = rng.uniform(0.5, 2.0, size=shape)
    net = nn.UNet(p, levels, c0, cin, alpha=0.1)
    loss, grads, _ = net.loss_and_grads(x, tgt, m)
    flat = nn.flatten(p, levels, c0, cin)
    gflat = nn.flatten(grads, levels, c0, cin)
    idx = rng.choice(flat.size, size=min(flat.size, 160), replace=False)
    # central differences at h = 1e-6 carry ~1e-10 |loss| / h of rounding and
    # O(h^2) truncation; a wrong term in the backward pass is off by O(1)
    h = 1e-6
    worst = 0.0
    for i in idx:
        fp = flat.copy()
        fp[i] += h
        lp = nn.UNet(nn.unflatten(fp, levels, c0, cin), levels, c0, cin, 0.1).loss_and_grads(x, tgt, m)[0]
        fp[i] -= 2 * h
        lm = nn.UNet(nn.unflatten(fp, levels, c0, cin), levels, c0, cin, 0.1).loss_and_grads(x, tgt, m)[0]
        fd = (lp - lm) / (2 * h)
        worst = max(worst, abs(fd - gflat[i]) / max(1e-3, abs(gflat[i])))
    assert worst < 1e-5, worst


def test_unet_matches_torch_autograd():
    """The same network assembled from torch's CPU layers, differentiated by autograd."""
    levels, c0, cin = 3, 4, 2
    p = _random_params(levels, c0, cin, seed=7, scale=0.15)
    rng = np.random.default_rng(8)
    x = rng.normal(size=(2, 8, 8, 8, cin))
    tgt = rng.normal(size=(2, 8, 8, 8))
    loss, grads, out = nn.UNet(p, levels, c0, cin, 0.01).loss_and_grads(x, tgt)
    tp = {k: torch.tensor(v, requires_grad=True) for k, v in p.items()}
    xt = _ncdhw(x)

    def conv(name, h):
        co, _, ci = tp[name + ".w"].shape
        wt = tp[name + ".w"].reshape(co, 3, 3, 3, ci).permute(0, 4, 1, 2, 3)
        return F.leaky_relu(F.conv3d(h, wt, tp[name + ".b"], padding=1), 0.01)

    skips, h = [], xt
    for l in range(levels):
        if l:
            h = F.avg_pool3d(h, 2)
        h = conv(f"enc{l}b", conv(f"enc{l}a", h))
        skips.append(h)
    for l in range(levels - 2, -1, -1):
        h = torch.cat([skips[l], F.interpolate(h, scale_factor=2, mode="nearest")], dim=1)
        h = conv(f"dec{l}b", conv(f"dec{l}a", h))
    o = xt[:, 0] + torch.einsum("bcdhw,c->bdhw", h, tp["head.w"]) + tp["head.b"][0]
    lt = ((o - torch.from_numpy(tgt)) ** 2).mean()
    lt.backward()
    np.testing.assert_allclose(out, o.detach().numpy(), rtol=1e-12, atol=1e-12)
    assert abs(loss - lt.item()) <= 1e-12 * abs(loss)
    for k in p:
        g = tp[k].grad.numpy()
        np.testing.assert_allclose(grads[k], g, rtol=0, atol=1e-11 * np.abs(g).max(), err_msg=k)


def test_unet_identity_wiring_closed_form():
    """With alpha = 1 and centre-tap identity kernels the encoder passes x
    through; a decoder that selects the skip half returns the level-0 input,
    one that selects the up half returns up(pool(x))."""
    levels, c0, cin = 2, 2, 2
    rng = np.random.default_rng(9)
    x = rng.normal(size=(1, 4, 6, 8, cin))

    def ident(co, ci, off=0):
        w = np.zeros((co, 27, ci))
        for c in range(co):
            w[c, 13, c + off] = 1.0
        return w

    def params(off):
        p = {n: np.zeros(s) for n, s in nn.param_shapes(levels, c0, cin)}
        p["enc0a.w"] = ident(2, 2)
        p["enc0b.w"] = ident(2, 2)
        p["enc1a.w"] = np.pad(ident(2, 2), ((0, 2), (0, 0), (0, 0)))   # channels 2, 3 stay 0
        p["enc1b.w"] = ident(4, 4)
        p["dec0a.w"] = ident(2, 6, off)
        p["dec0b.w"] = ident(2, 2)
        p["head.w"] = np.array([1.0, 0.0])
        return p

    out_skip, _ = nn.UNet(params(0), levels, c0, cin, alpha=1.0).forward(x)
    np.testing.assert_allclose(out_skip, 2 * x[..., 0], atol=1e-14)
    out_up, _ = nn.UNet(params(2), levels, c0, cin, alpha=1.0).forward(x)
    np.testing.assert_allclose(out_up, x[..., 0] + nn.up2(nn.pool2(x))[..., 0], atol=1e-14)


def test_bf16_rounding_matches_torch():
    """The storage rounding is round-to-nearest-even to bf16 (torch's cast)."""
    rng = np.random.default_rng(10)
    a = np.concatenate([rng.normal(scale=10.0 ** rng.uniform(-20, 20, 4000)),
                        [0.0, -0.0, 1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -(1.0 + 2 ** -8), 65504.0]])
    a = a.astype(np.float32)
    ref = torch.from_numpy(a).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(nn.bf16(a), ref)
    # ties: 1 + 2^-8 lies halfway between 1 and 1 + 2^-7 and rounds to the even 1
    assert nn.bf16(np.array([1.0 + 2 ** -8]))[0] == 1.0
    assert nn.bf16(np.array([1.0 + 3 * 2 ** -8]))[0] == 1.0 + 2 ** -6


def test_bf16_storage_is_a_small_perturbation_off_the_residual():
    """bf16 storage moves the output by a small fraction of the head's
    contribution, and never touches the residual path."""
    levels, c0, cin = 2, 2, 2
    rng = np.random.default_rng(11)
    x = rng.normal(size=(1, 4, 4, 4, cin))
    p = {n: rng.normal(scale=0.3, size=s) for n, s in nn.param_shapes(levels, c0, cin)}
    o1, _ = nn.UNet(p, levels, c0, cin, 0.01, bf16_storage=True).forward(x)
    o0, _ = nn.UNet(p, levels, c0, cin, 0.01).forward(x)
    assert 0 < np.abs(o1 - o0).max() < 0.05 * np.abs(o0 - x[..., 0]).max()
    # the residual is never rounded
    q = dict(p)
    q["head.w"] = np.zeros(c0)
    q["head.b"] = np.zeros(1)
    o2, _ = nn.UNet(q, levels, c0, cin, 0.01, bf16_storage=True).forward(x)
    np.testing.assert_array_equal(o2, x[..., 0])
