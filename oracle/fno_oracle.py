"""FP64 CPU oracle of the warm-start surrogate network (test infrastructure).

TEST INFRASTRUCTURE ONLY: used by the tests to check the forward pass and
the gradients of the GPU implementation; never by the product path, with
which it shares no code.  Plain PyTorch CPU operations in float64, with the
Fourier transforms written out as complex exponentials and the gradients
taken by autograd.

Network (a Fourier neural operator on an S x S grid, channel-last):
  input features a (5 channels)
  h_0 = a W_lift + b_lift
  for l = 0 .. L-1:
      s_l   = spectral_l(h_l) + h_l W_l + b_l
      h_l+1 = GELU(s_l)        (identity for the last layer)
  out = GELU(h_L P_1 + c_1) P_2 + c_2      (4 channels)
spectral(h)[b, y, x, o] = (1/S^2) sum_{ky in K_y} sum_{kx < m} alpha(kx)
      Re{ Z[b, ky, kx, o] exp(+2 pi i (ky y + kx x) / S) },
  Z[b, ky, kx, o] = sum_c H[b, ky, kx, c] R[ky, kx, c, o]  (complex R),
  H[b, ky, kx, c] = sum_{y, x} h[b, y, x, c] exp(-2 pi i (ky y + kx x) / S),
  K_y = {0 .. m-1} + {S-m .. S-1}, alpha(0) = 1, alpha(kx > 0) = 2.
GELU(x) = x (1 + erf(x / sqrt 2)) / 2.
"""
from __future__ import annotations

import math

import torch


def gelu(x):
    return 0.5 * x * (1.0 + torch.erf(x / math.sqrt(2.0)))


def ky_modes(S: int, m: int):
    return list(range(m)) + list(range(S - m, S))


def spectral(h, R_re, R_im, m):
    """h: (B, S, S, C) float64; R_re, R_im: (2m, m, C, O)."""
    B, S, _, C = h.shape
    ky = torch.tensor(ky_modes(S, m), dtype=torch.float64)
    kx = torch.arange(m, dtype=torch.float64)
    pos = torch.arange(S, dtype=torch.float64)
    Ey = torch.exp(-2j * math.pi * torch.outer(ky, pos) / S)   # (2m, S) over y
    Ex = torch.exp(-2j * math.pi * torch.outer(kx, pos) / S)   # (m, S) over x
    hc = h.to(torch.complex128)
    H = torch.einsum("ay,bx,nyxc->nabc", Ey, Ex, hc)           # (B, 2m, m, C)
    R = torch.complex(R_re, R_im)
    Z = torch.einsum("nabc,abco->nabo", H, R)
    alpha = torch.ones(m, dtype=torch.float64)
    alpha[1:] = 2.0
    Iy = torch.exp(2j * math.pi * torch.outer(pos, ky) / S)    # (S, 2m)
    Ix = torch.exp(2j * math.pi * torch.outer(pos, kx) / S) * alpha  # (S, m)
    z = torch.einsum("ya,xb,nabo->nyxo", Iy, Ix, Z).real / (S * S)
    return z


def forward(params: dict, a, m: int):
    """params: dict of float64 tensors (see ``init_params``); a: (B, S, S, 5)."""
    h = a @ params["W_lift"] + params["b_lift"]
    L = len([k for k in params if k.startswith("R_re_")])
    for l in range(L):
        s = spectral(h, params[f"R_re_{l}"], params[f"R_im_{l}"], m) + h @ params[f"W_{l}"] + params[f"b_{l}"]
        h = gelu(s) if l < L - 1 else s
    q = gelu(h @ params["P1"] + params["c1"])
    return q @ params["P2"] + params["c2"]


def loss_and_grads(params: dict, a, target, m: int):
    """Mean-squared error and its gradients with respect to every parameter."""
    p = {k: v.detach().clone().requires_grad_(True) for k, v in params.items()}
    out = forward(p, a, m)
    loss = ((out - target) ** 2).mean()
    loss.backward()
    return out.detach(), float(loss.detach()), {k: v.grad.detach() for k, v in p.items()}
