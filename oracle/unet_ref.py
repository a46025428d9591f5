"""Plain CPU float64 reference of the warm-start network (TEST INFRASTRUCTURE).

Only the tests and the smoke check use this module.  It restates the network
the HIP library implements -- 3^3 periodic convolutions, 2^3 mean pooling,
nearest-neighbour upsampling, channel concatenation, ReLU, a 1x1 head and a
mean-squared-error loss against u / 5 -- with plain PyTorch CPU operations in
float64; gradients come from autograd.  The parameter vector has the
library's layout: for each of the 10 convolutions, weights [27][Cout][Cin]
(tap t = (dz+1)*9 + (dy+1)*3 + (dx+1)) then biases [Cout]; then the head's 16
weights and its bias.  Input features: asinh(delta)/4, (a - 0.75)*4,
(log10|f_R0| + 5.5)/1.5 and 13 zero channels.
"""
from __future__ import annotations

import math

import torch
import torch.nn.functional as F

LAYERS = [(16, 16), (16, 16), (16, 32), (32, 32), (32, 64), (64, 64), (96, 32), (32, 32), (48, 16), (16, 16)]
U_SCALE = 5.0


def num_params() -> int:
    return sum(27 * ci * co + co for ci, co in LAYERS) + 17


def unpack(p: torch.Tensor):
    """Split the flat parameter vector into torch conv weights [Cout, Cin, 3, 3, 3] and biases."""
    out, off = [], 0
    for ci, co in LAYERS:
        w = p[off:off + 27 * ci * co].reshape(27, co, ci)
        off += 27 * ci * co
        b = p[off:off + co]
        off += co
        # tap t = kd*9 + kh*3 + kw with kd <-> z, kh <-> y, kw <-> x
        wt = w.permute(1, 2, 0).reshape(co, ci, 3, 3, 3)
        out.append((wt, b))
    head_w = p[off:off + 16]
    head_b = p[off + 16]
    return out, head_w, head_b


def conv3d_periodic(x: torch.Tensor, w: torch.Tensor, b=None) -> torch.Tensor:
    """x [B, C, D, H, W] with periodic boundaries, w [Cout, Cin, 3, 3, 3] (cross-correlation)."""
    return F.conv3d(F.pad(x, (1, 1, 1, 1, 1, 1), mode="circular"), w, b)


def features(delta: torch.Tensor, cond) -> torch.Tensor:
    """delta [B, S, S, S] -> [B, 16, S, S, S]."""
    B = delta.shape[0]
    x = torch.zeros((B, 16) + tuple(delta.shape[1:]), dtype=torch.float64)
    x[:, 0] = torch.asinh(delta) * 0.25
    for b in range(B):
        a, fr0 = cond[b]
        x[b, 1] = (a - 0.75) * 4.0
        x[b, 2] = (math.log10(fr0) + 5.5) / 1.5
    return x


def forward(p: torch.Tensor, x: torch.Tensor) -> torch.Tensor:
    """Network output y [B, S, S, S] (= predicted u / 5) for input features x."""
    convs, hw, hb = unpack(p)
    r = lambda t, i: F.relu(conv3d_periodic(t, *convs[i]))
    s1 = r(r(x, 0), 1)
    s2 = r(r(F.avg_pool3d(s1, 2), 2), 3)
    h3 = r(r(F.avg_pool3d(s2, 2), 4), 5)
    up = lambda t: t.repeat_interleave(2, 2).repeat_interleave(2, 3).repeat_interleave(2, 4)
    h4 = r(r(torch.cat([up(h3), s2], dim=1), 6), 7)
    h5 = r(r(torch.cat([up(h4), s1], dim=1), 8), 9)
    return torch.einsum("bcdhw,c->bdhw", h5, hw) + hb


def loss(p: torch.Tensor, x: torch.Tensor, u: torch.Tensor) -> torch.Tensor:
    return ((forward(p, x) - u / U_SCALE) ** 2).mean()


def loss_and_grad(p: torch.Tensor, x: torch.Tensor, u: torch.Tensor):
    q = p.detach().clone().requires_grad_(True)
    L = loss(q, x, u)
    (g,) = torch.autograd.grad(L, q)
    return L.item(), g


def adam_step(p, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One bias-corrected Adam update (Kingma & Ba); returns new (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (torch.sqrt(vh) + eps), m, v
