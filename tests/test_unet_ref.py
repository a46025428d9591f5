"""Pins of the CPU float64 network reference (no GPU): autograd gradients
against central finite differences, the periodic convolution against an
explicit sum over taps, and the layer/parameter layout."""
import math

import numpy as np
import torch

from oracle import unet_ref as U


def test_param_count_matches_the_stated_architecture():
    # 3-level U-Net with 16/32/64 channels, 10 3^3 convolutions and a 1x1 head
    ci_co = [16 * 16, 16 * 16, 16 * 32, 32 * 32, 32 * 64, 64 * 64, 96 * 32, 32 * 32, 48 * 16, 16 * 16]
    assert U.num_params() == 27 * sum(ci_co) + (16 + 16 + 32 + 32 + 64 + 64 + 32 + 32 + 16 + 16) + 17 == 359761


def test_periodic_conv_equals_explicit_tap_sum():
    g = torch.Generator().manual_seed(0)
    x = torch.randn((1, 3, 4, 4, 4), generator=g, dtype=torch.float64)
    w = torch.randn((2, 3, 3, 3, 3), generator=g, dtype=torch.float64)
    y = U.conv3d_periodic(x, w)
    ref = torch.zeros_like(y)
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                xs = torch.roll(x, shifts=(-dz, -dy, -dx), dims=(2, 3, 4))  # xs[z] = x[z + dz]
                ref += torch.einsum("bcdhw,oc->bodhw", xs, w[:, :, dz + 1, dy + 1, dx + 1])
    assert torch.allclose(y, ref, atol=1e-12)


def test_autograd_matches_finite_differences():
    g = torch.Generator().manual_seed(1)
    p = torch.randn(U.num_params(), generator=g, dtype=torch.float64) * 0.05
    delta = torch.exp(torch.randn((1, 8, 8, 8), generator=g, dtype=torch.float64)) - 1
    x = U.features(delta, [(0.8, 1e-5)])
    u = -torch.rand((1, 8, 8, 8), generator=g, dtype=torch.float64) * 3
    L, grad = U.loss_and_grad(p, x, u)
    rng = np.random.default_rng(2)
    idx = rng.choice(U.num_params(), 12, replace=False)
    for i in idx:
        e = torch.zeros_like(p)
        e[i] = 1e-6
        fd = (U.loss(p + e, x, u) - U.loss(p - e, x, u)).item() / 2e-6
        assert abs(fd - grad[i].item()) <= 1e-7 * max(1.0, abs(fd)) + 1e-9


def test_adam_first_step_is_signed_lr():
    p = torch.tensor([1.0, -2.0, 3.0], dtype=torch.float64)
    gr = torch.tensor([0.5, -4.0, 1e-3], dtype=torch.float64)
    pn, m, v = U.adam_step(p, gr, torch.zeros(3, dtype=torch.float64), torch.zeros(3, dtype=torch.float64), 1, 0.01)
    # first bias-corrected step: m_hat = g, v_hat = g^2 -> p - lr g / (|g| + eps)
    assert torch.allclose(pn, p - 0.01 * gr / (gr.abs() + 1e-8), atol=1e-15)
