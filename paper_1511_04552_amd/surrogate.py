"""Warm-start surrogate: a Fourier neural operator mapping the cavity
parameters (Ra, phi0, d_p) and a coordinate grid to near-steady fields
(u, v, theta, phi).  The lattice Boltzmann solver starts from its prediction
(``Cavity.load_fields``) and still runs to its own convergence criterion, so
the surrogate changes the time to steady state, never the converged answer.

Every operation runs in the library's kernels (``include/mclbm_nn.h``): the
matrix products (the Fourier transforms are written as products with cosine
and sine matrices) on BF16 matrix cores with FP32 accumulation, and the bias,
activation, loss and optimiser steps as elementwise kernels.  PyTorch only
owns the device buffers.

Network on an S x S grid, channel-last activations (B, S, S, C):
  h_0 = a W_lift + b_lift                         (a: 5 input features)
  s_l = spectral_l(h_l) + h_l W_l + b_l,  h_l+1 = GELU(s_l) (identity last)
  out = GELU(h_L P1 + c1) P2 + c2                 (nout output fields)
spectral(h) = (1/S^2) sum_{ky in K_y, kx < m} alpha(kx)
              Re{ (H R)(ky, kx) e^{+2 pi i (ky y + kx x)/S} },
H(ky, kx) = sum_{y,x} h e^{-2 pi i (ky y + kx x)/S}, K_y = {0..m-1} u
{S-m..S-1}, alpha(0) = 1, alpha(kx > 0) = 2, R complex per mode.
"""
from __future__ import annotations

import ctypes
import math

import numpy as np

from . import _check, lib

GELU, IDENT = 1, 0


def _p(t, off=0):
    if not t.is_contiguous():
        raise ValueError("kernel operands must be contiguous")
    return ctypes.c_void_p(t.data_ptr() + t.element_size() * int(off))


class _Ops:
    """Kernel calls on one stream."""

    def __init__(self, torch, stream):
        self.torch = torch
        self.s = ctypes.c_void_p(stream.cuda_stream)

    def gemm(self, ta, tb, M, N, K, alpha, A, aoff, lda, sa1, sa2, B, boff, ldb, sb1, sb2,
             beta, C, coff, ldc, sc1, sc2, nb1=1, nb2=1):
        _check(lib().mclbm_nn_gemm(ta, tb, M, N, K, alpha, _p(A, aoff), lda, sa1, sa2,
                                   _p(B, boff), ldb, sb1, sb2, beta, _p(C, coff), ldc, sc1, sc2,
                                   nb1, nb2, self.s))

    def bias_act(self, y, bias, rows, cols, act, pre=None):
        _check(lib().mclbm_nn_bias_act(_p(y), None if bias is None else _p(bias), rows, cols, act,
                                       None if pre is None else _p(pre), self.s))

    def act_backward(self, dy, pre, act):
        _check(lib().mclbm_nn_act_backward(_p(dy), _p(pre), dy.numel(), act, self.s))

    def colsum(self, dy, db, rows, cols, scratch, beta=0.0):
        _check(lib().mclbm_nn_colsum(_p(dy), _p(db), rows, cols, beta, _p(scratch), self.s))

    def mse(self, y, t, dy, scratch, loss):
        _check(lib().mclbm_nn_mse(_p(y), _p(t), _p(dy), y.numel(), _p(scratch), _p(loss), self.s))

    def adamw(self, w, g, m, v, lr, b1, b2, eps, wd, t):
        _check(lib().mclbm_nn_adamw(_p(w), _p(g), _p(m), _p(v), w.numel(), lr, b1, b2, eps, wd, t, self.s))


def dft_matrices(S: int, m: int) -> dict:
    """Real matrices of the truncated transforms (float32)."""
    x = np.arange(S)
    kx = np.arange(m)
    ky = np.array(list(range(m)) + list(range(S - m, S)))
    tx = 2 * np.pi * np.outer(kx, x) / S            # (m, S)
    ty = 2 * np.pi * np.outer(ky, x) / S            # (2m, S)
    Gc, Gs = np.cos(ty), np.sin(ty)
    G = np.block([[Gc, Gs], [-Gs, Gc]])            # (4m, 2S): forward along y
    Hm = np.block([[Gc.T, -Gs.T], [Gs.T, Gc.T]])   # (2S, 4m): inverse along y
    alpha = np.where(kx == 0, 1.0, 2.0)
    Ec = (np.cos(tx) * alpha[:, None]).T / (S * S)  # (S, m): inverse along x, real part
    Es = (-np.sin(tx) * alpha[:, None]).T / (S * S)
    mats = {"Fc": np.cos(tx), "Fs": -np.sin(tx), "G": G, "Hm": Hm, "Ec": Ec, "Es": Es}
    return {k: np.ascontiguousarray(v, dtype=np.float32) for k, v in mats.items()}


class FNO:
    """Fourier neural operator on the GPU (training and inference)."""

    def __init__(self, S=64, C=32, m=12, L=4, Q=64, B=16, seed=0, device="cuda", stream=None, nout=5):
        import torch
        self.torch = torch
        self.S, self.C, self.m, self.L, self.Q, self.B = S, C, m, L, Q, B
        self.nout = nout
        self.M2 = 2 * m
        self.nq = self.M2 * m
        self.dev = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.dev)
        self.ops = _Ops(torch, self.stream)
        rng = np.random.default_rng(seed)
        f32 = lambda a: torch.tensor(np.ascontiguousarray(a, dtype=np.float32), device=self.dev)
        self.mats = {k: f32(v) for k, v in dft_matrices(S, m).items()}
        p = {"W_lift": rng.normal(0, 1 / math.sqrt(5), (5, C)), "b_lift": np.zeros(C)}
        for l in range(L):
            sc = 1.0 / (C * C)
            p[f"R_re_{l}"] = sc * rng.uniform(0, 1, (self.M2, m, C, C))
            p[f"R_im_{l}"] = sc * rng.uniform(0, 1, (self.M2, m, C, C))
            p[f"W_{l}"] = rng.normal(0, 1 / math.sqrt(C), (C, C))
            p[f"b_{l}"] = np.zeros(C)
        p["P1"] = rng.normal(0, 1 / math.sqrt(C), (C, Q))
        p["c1"] = np.zeros(Q)
        p["P2"] = rng.normal(0, 1 / math.sqrt(Q), (Q, nout))
        p["c2"] = np.zeros(nout)
        self.params = {k: f32(v) for k, v in p.items()}
        self.grads = {k: torch.zeros_like(v) for k, v in self.params.items()}
        self.adam_m = {k: torch.zeros_like(v) for k, v in self.params.items()}
        self.adam_v = {k: torch.zeros_like(v) for k, v in self.params.items()}
        self.adam_t = 0
        self._alloc(B)

    # ---- buffers --------------------------------------------------------
    def _alloc(self, B):
        torch, S, C, m, Q = self.torch, self.S, self.C, self.m, self.Q
        z = lambda *shape: torch.zeros(*shape, dtype=torch.float32, device=self.dev)
        self.B = B
        rows = B * S * S
        self.h = [z(rows, C) for _ in range(self.L + 1)]        # layer inputs / outputs
        self.pre = [z(rows, C) for _ in range(self.L)]          # pre-activations
        self.Y = [z(B, 2, self.nq, C) for _ in range(self.L)]    # spectra after the y-transform
        self.X = z(B, 2, S, m, C)
        self.Z = z(B, 2, self.nq, C)
        self.W = z(B, 2, S, m, C)
        self.qpre, self.q = z(rows, Q), z(rows, Q)
        self.out = z(rows, self.nout)
        self.dout, self.dq = z(rows, self.nout), z(rows, Q)
        self.dh, self.dh2 = z(rows, C), z(rows, C)
        self.dX, self.dZ, self.dW, self.dY = z(B, 2, S, m, C), z(B, 2, self.nq, C), z(B, 2, S, m, C), z(B, 2, self.nq, C)
        ncol = max(C, Q, self.nout)
        # K split of the weight gradients: slices of at least 256 rows
        self.ksplit = 1
        while self.ksplit < 256 and rows % (2 * self.ksplit) == 0 and rows // (2 * self.ksplit) >= 256:
            self.ksplit *= 2
        wmax = max(C * C, C * Q, Q * self.nout, 5 * C)
        self.ws = z(self.ksplit * wmax)
        self.cs_scratch = z(max(int(lib().mclbm_nn_colsum_scratch(rows, ncol)),
                                int(lib().mclbm_nn_colsum_scratch(self.ksplit, wmax))))
        self.mse_scratch = torch.zeros(int(lib().mclbm_nn_mse_scratch(rows * self.nout)), dtype=torch.float64,
                                       device=self.dev)
        self.loss_dev = torch.zeros(1, dtype=torch.float64, device=self.dev)

    # ---- weight gradients: G = op(X)^T Y over all rows, split over K ----
    def _wgrad(self, X, ldx, Y, ldy, M, N, G):
        """G (M x N) = X^T Y for X (rows x M, row stride ldx) and Y (rows x N):
        the rows (the long K dimension) are split into ``ksplit`` slices
        computed as one batched GEMM into a workspace, whose slices are then
        summed in a fixed order by the column-sum kernel."""
        rows = self.B * self.S * self.S
        ks = self.ksplit
        o = self.ops
        o.gemm(1, 0, M, N, rows // ks, 1.0, X, 0, ldx, (rows // ks) * ldx, 0, Y, 0, ldy, (rows // ks) * ldy, 0,
               0.0, self.ws, 0, N, M * N, 0, ks, 1)
        o.colsum(self.ws, G, ks, M * N, self.cs_scratch)

    # ---- spectral layer -------------------------------------------------
    def _spectral_forward(self, h, l, out):
        o, S, C, m, nq, B = self.ops, self.S, self.C, self.m, self.nq, self.B
        M, SmC, mC = self.mats, S * m * C, m * C
        # x-transform, per (b, y): X_re = Fc h[b, y], X_im = Fs h[b, y]
        for ri, F in ((0, M["Fc"]), (1, M["Fs"])):
            o.gemm(0, 0, m, C, S, 1.0, F, 0, S, 0, 0, h, 0, C, S * S * C, S * C,
                   0.0, self.X, ri * SmC, C, 2 * SmC, mC, B, S)
        # y-transform, per b: [Y_re; Y_im] = G [X_re; X_im]
        Y = self.Y[l]
        o.gemm(0, 0, 2 * self.M2, mC, 2 * S, 1.0, M["G"], 0, 2 * S, 0, 0, self.X, 0, mC, 2 * SmC, 0,
               0.0, Y, 0, mC, 2 * nq * C, 0, B, 1)
        # complex mode mixing, per mode q: Z = Y R
        Rr, Ri = self.params[f"R_re_{l}"], self.params[f"R_im_{l}"]
        ld = 2 * nq * C
        for (yi, Rt, zi, alpha, beta) in ((0, Rr, 0, 1.0, 0.0), (1, Ri, 0, -1.0, 1.0),
                                          (0, Ri, 1, 1.0, 0.0), (1, Rr, 1, 1.0, 1.0)):
            o.gemm(0, 0, B, C, C, alpha, Y, yi * nq * C, ld, C, 0, Rt, 0, C, C * C, 0,
                   beta, self.Z, zi * nq * C, ld, C, 0, nq, 1)
        # inverse y-transform, per b: [W_re; W_im] = Hm [Z_re; Z_im]
        o.gemm(0, 0, 2 * S, mC, 2 * self.M2, 1.0, M["Hm"], 0, 2 * self.M2, 0, 0, self.Z, 0, mC, 2 * nq * C, 0,
               0.0, self.W, 0, mC, 2 * SmC, 0, B, 1)
        # inverse x-transform (real part), per (b, y): out = Ec W_re + Es W_im
        for ri, E, beta in ((0, M["Ec"], 0.0), (1, M["Es"], 1.0)):
            o.gemm(0, 0, S, C, m, 1.0, E, 0, m, 0, 0, self.W, ri * SmC, C, 2 * SmC, mC,
                   beta, out, 0, C, S * S * C, S * C, B, S)

    def _spectral_backward(self, l, dout, dh):
        """dh += spectral_l^T(dout); accumulates dR_re, dR_im."""
        o, S, C, m, nq, B = self.ops, self.S, self.C, self.m, self.nq, self.B
        M, SmC, mC = self.mats, S * m * C, m * C
        for ri, E in ((0, M["Ec"]), (1, M["Es"])):
            o.gemm(1, 0, m, C, S, 1.0, E, 0, m, 0, 0, dout, 0, C, S * S * C, S * C,
                   0.0, self.dW, ri * SmC, C, 2 * SmC, mC, B, S)
        o.gemm(1, 0, 2 * self.M2, mC, 2 * S, 1.0, M["Hm"], 0, 2 * self.M2, 0, 0, self.dW, 0, mC, 2 * SmC, 0,
               0.0, self.dZ, 0, mC, 2 * nq * C, 0, B, 1)
        Y = self.Y[l]
        Rr, Ri = self.params[f"R_re_{l}"], self.params[f"R_im_{l}"]
        gRr, gRi = self.grads[f"R_re_{l}"], self.grads[f"R_im_{l}"]
        ld = 2 * nq * C
        # dY_re = dZ_re Rr^T + dZ_im Ri^T ; dY_im = -dZ_re Ri^T + dZ_im Rr^T
        for (zi, Rt, yi, alpha, beta) in ((0, Rr, 0, 1.0, 0.0), (1, Ri, 0, 1.0, 1.0),
                                          (0, Ri, 1, -1.0, 0.0), (1, Rr, 1, 1.0, 1.0)):
            o.gemm(0, 1, B, C, C, alpha, self.dZ, zi * nq * C, ld, C, 0, Rt, 0, C, C * C, 0,
                   beta, self.dY, yi * nq * C, ld, C, 0, nq, 1)
        # dRr = Y_re^T dZ_re + Y_im^T dZ_im ; dRi = -Y_im^T dZ_re + Y_re^T dZ_im
        for (yi, zi, G_, alpha, beta) in ((0, 0, gRr, 1.0, 0.0), (1, 1, gRr, 1.0, 1.0),
                                          (1, 0, gRi, -1.0, 0.0), (0, 1, gRi, 1.0, 1.0)):
            o.gemm(1, 0, C, C, B, alpha, Y, yi * nq * C, ld, C, 0, self.dZ, zi * nq * C, ld, C, 0,
                   beta, G_, 0, C, C * C, 0, nq, 1)
        o.gemm(1, 0, 2 * S, mC, 2 * self.M2, 1.0, M["G"], 0, 2 * S, 0, 0, self.dY, 0, mC, 2 * nq * C, 0,
               0.0, self.dX, 0, mC, 2 * SmC, 0, B, 1)
        for ri, F in ((0, M["Fc"]), (1, M["Fs"])):
            o.gemm(1, 0, S, C, m, 1.0, F, 0, S, 0, 0, self.dX, ri * SmC, C, 2 * SmC, mC,
                   1.0, dh, 0, C, S * S * C, S * C, B, S)

    # ---- whole network ----------------------------------------------------
    def forward(self, a):
        """a: (B, S, S, 5) float32 device tensor.  Returns (B, S, S, nout)."""
        o, C, Q = self.ops, self.C, self.Q
        rows = self.B * self.S * self.S
        a = a.reshape(rows, 5)
        self._a = a
        P = self.params
        o.gemm(0, 0, rows, C, 5, 1.0, a, 0, 5, 0, 0, P["W_lift"], 0, C, 0, 0, 0.0, self.h[0], 0, C, 0, 0)
        o.bias_act(self.h[0], P["b_lift"], rows, C, IDENT)
        for l in range(self.L):
            s = self.h[l + 1]
            self._spectral_forward(self.h[l], l, s)
            o.gemm(0, 0, rows, C, C, 1.0, self.h[l], 0, C, 0, 0, P[f"W_{l}"], 0, C, 0, 0, 1.0, s, 0, C, 0, 0)
            o.bias_act(s, P[f"b_{l}"], rows, C, GELU if l < self.L - 1 else IDENT, self.pre[l])
        o.gemm(0, 0, rows, Q, C, 1.0, self.h[self.L], 0, C, 0, 0, P["P1"], 0, Q, 0, 0, 0.0, self.q, 0, Q, 0, 0)
        o.bias_act(self.q, P["c1"], rows, Q, GELU, self.qpre)
        no = self.nout
        o.gemm(0, 0, rows, no, Q, 1.0, self.q, 0, Q, 0, 0, P["P2"], 0, no, 0, 0, 0.0, self.out, 0, no, 0, 0)
        o.bias_act(self.out, P["c2"], rows, no, IDENT)
        return self.out.reshape(self.B, self.S, self.S, no)

    def backward(self, target):
        """MSE against target (B, S, S, nout): fills self.grads, returns the loss
        (device tensor, FP64)."""
        o, C, Q = self.ops, self.C, self.Q
        rows = self.B * self.S * self.S
        P, G = self.params, self.grads
        no = self.nout
        o.mse(self.out, target.reshape(rows, no), self.dout, self.mse_scratch, self.loss_dev)
        o.colsum(self.dout, G["c2"], rows, no, self.cs_scratch)
        self._wgrad(self.q, Q, self.dout, no, Q, no, G["P2"])
        o.gemm(0, 1, rows, Q, no, 1.0, self.dout, 0, no, 0, 0, P["P2"], 0, no, 0, 0, 0.0, self.dq, 0, Q, 0, 0)
        o.act_backward(self.dq, self.qpre, GELU)
        o.colsum(self.dq, G["c1"], rows, Q, self.cs_scratch)
        self._wgrad(self.h[self.L], C, self.dq, Q, C, Q, G["P1"])
        dh = self.dh
        o.gemm(0, 1, rows, C, Q, 1.0, self.dq, 0, Q, 0, 0, P["P1"], 0, Q, 0, 0, 0.0, dh, 0, C, 0, 0)
        for l in reversed(range(self.L)):
            if l < self.L - 1:
                o.act_backward(dh, self.pre[l], GELU)
            o.colsum(dh, G[f"b_{l}"], rows, C, self.cs_scratch)
            self._wgrad(self.h[l], C, dh, C, C, C, G[f"W_{l}"])
            dprev = self.dh2
            o.gemm(0, 1, rows, C, C, 1.0, dh, 0, C, 0, 0, P[f"W_{l}"], 0, C, 0, 0, 0.0, dprev, 0, C, 0, 0)
            self._spectral_backward(l, dh, dprev)
            self.dh, self.dh2 = dprev, dh
            dh = self.dh
        o.colsum(dh, G["b_lift"], rows, C, self.cs_scratch)
        self._wgrad(self._a, 5, dh, C, 5, C, G["W_lift"])
        return self.loss_dev

    def step(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, wd=1e-4):
        self.adam_t += 1
        for k, w in self.params.items():
            self.ops.adamw(w, self.grads[k], self.adam_m[k], self.adam_v[k], lr, b1, b2, eps, wd, self.adam_t)

    # ---- persistence -----------------------------------------------------
    def state(self) -> dict:
        return {k: v.detach().cpu().numpy() for k, v in self.params.items()}

    def load_state(self, st: dict) -> None:
        for k, v in st.items():
            self.params[k].copy_(self.torch.tensor(v, dtype=self.torch.float32))


# ==========================================================================
# Warm start: data, training, prediction, loading
# ==========================================================================
TARGETS = ("rho_f", "phi", "theta", "ux_ns", "uy_ns")
NCH = 5  # u, v, theta, phi, fluid-density deviation


def velocity_scale(cfg: dict) -> float:
    """Convective velocity scale alpha sqrt(Ra) / H in lattice units: it
    makes the steady velocities of the whole Ra range O(0.1 - 0.3)."""
    from . import derive_constants
    d = derive_constants(**_cavity_kw(cfg))
    return d["alpha_L"] * math.sqrt(max(cfg["Ra"], 1.0)) / cfg["nx"]


def features(cases, S: int) -> np.ndarray:
    """Network input (n, S, S, 5): scaled log10 Ra, phi0, d_p and the cell
    coordinates in [-1, 1]."""
    n = len(cases)
    a = np.zeros((n, S, S, 5), np.float32)
    xs = 2.0 * (np.arange(S) + 0.5) / S - 1.0
    for k, c in enumerate(cases):
        a[k, :, :, 0] = (math.log10(max(c["Ra"], 1.0)) - 4.5) / 1.5
        a[k, :, :, 1] = (c["phi0"] - 0.025) / 0.025
        a[k, :, :, 2] = (c["dp_nm"] - 55.0) / 45.0
        a[k, :, :, 3] = xs[None, :]
        a[k, :, :, 4] = xs[:, None]
    return a


def density_scale(cfg: dict) -> float:
    """Hydrostatic density scale of the buoyancy: the lattice pressure
    c_s^2 delta rho balances rho G_L theta over the height, so
    delta rho ~ 3 G_L nx."""
    from . import derive_constants
    d = derive_constants(**_cavity_kw(cfg))
    return max(3.0 * d["G_L"] * cfg["nx"], 1e-12)


def nondimensional(moments: dict, cfg: dict) -> np.ndarray:
    """(ny, nx, 5): u / U, v / U, theta, phi / phi0 - 1 (0 without
    particles), (rho_f~ - (1 - phi0)) / (3 G_L nx)."""
    U = velocity_scale(cfg)
    out = np.zeros(moments["theta"].shape + (NCH,), np.float32)
    out[..., 0] = moments["ux_ns"] / U
    out[..., 1] = moments["uy_ns"] / U
    out[..., 2] = moments["theta"]
    if cfg["phi0"] > 1e-4:
        out[..., 3] = moments["phi"] / cfg["phi0"] - 1.0
    out[..., 4] = (moments["rho_f"] - (1.0 - cfg["phi0"])) / density_scale(cfg)
    return out


def _cavity_kw(c: dict) -> dict:
    return {k: v for k, v in c.items() if k != "seed"}


def generate_dataset(cases, chunk: int = 2000, tol: float = 1e-6, max_steps: int = 2_000_000,
                     log=None):
    """Run the cases (square cavities of one side) to steady state as one
    batch with drop-out: a cavity leaves the batch when the relative change
    of u and theta over ``chunk`` steps is below ``tol``.  Returns the
    nondimensional fields (n, S, S, 5), the step counts and a converged
    mask."""
    from . import Batch
    b = Batch([_cavity_kw(c) for c in cases])
    n = len(cases)
    status = np.zeros(n, np.int32)
    steps = np.zeros(n, np.int64)
    b.residual(tol=0.0)
    t = 0
    while t < max_steps and (status == 0).any():
        b.step(chunk)
        t += chunk
        _, st = b.residual(tol=tol)
        newly = (status == 0) & (st != 0)
        steps[newly] = t
        status[newly] = st[newly]
        if log and (t // chunk) % 50 == 0:
            log(f"  t={t} converged {(status == 1).sum()}/{n} diverged {(status == 2).sum()}")
    fields = np.stack([nondimensional(b.members[k].moments(TARGETS), cases[k]) for k in range(n)])
    return fields, steps, status == 1


class WarmStart:
    """Learned initial condition: the FNO plus the per-channel
    standardisation of its targets."""

    def __init__(self, S=64, C=32, m=12, L=4, Q=64, B=16, seed=0, device="cuda"):
        self.S, self.B = S, B
        self.net = FNO(S=S, C=C, m=m, L=L, Q=Q, B=B, seed=seed, device=device, nout=NCH)
        self.torch = self.net.torch
        self.mean = np.zeros(NCH)
        self.std = np.ones(NCH)
        self.seed = seed

    def fit(self, cases, fields, epochs=100, lr=2e-3, lr_min=1e-4, wd=1e-5, weights=None, log=None):
        """AdamW on the mean-squared error of the standardised fields, with a
        cosine learning-rate schedule.  ``weights`` (one per channel) scale
        the standardised targets, i.e. weight the squared error of channel c
        by weights[c]^2: the temperature field decays slowest after a warm
        start, so its accuracy matters most.  Returns the loss per epoch."""
        torch = self.torch
        n = len(cases)
        if n < self.B:
            raise ValueError("need at least one batch of training cases")
        w = np.ones(NCH) if weights is None else np.asarray(weights, dtype=np.float64)
        self.mean = fields.reshape(-1, NCH).mean(0).astype(np.float64)
        self.std = np.maximum(fields.reshape(-1, NCH).std(0).astype(np.float64), 1e-6) / w
        y = ((fields - self.mean) / self.std).astype(np.float32)
        dev = self.net.dev
        X = torch.tensor(features(cases, self.S), device=dev)
        Y = torch.tensor(y, device=dev)
        rng = np.random.default_rng(self.seed)
        nb = n // self.B
        xb = torch.empty((self.B,) + tuple(X.shape[1:]), dtype=torch.float32, device=dev)
        yb = torch.empty((self.B,) + tuple(Y.shape[1:]), dtype=torch.float32, device=dev)
        total = epochs * nb
        hist = []
        it = 0
        for ep in range(epochs):
            perm = rng.permutation(n)
            acc = torch.zeros(1, dtype=torch.float64, device=dev)
            for j in range(nb):
                # the batch: device-to-device copies of whole samples
                for q, k in enumerate(perm[j * self.B:(j + 1) * self.B]):
                    xb[q].copy_(X[int(k)])
                    yb[q].copy_(Y[int(k)])
                self.net.forward(xb)
                acc += self.net.backward(yb)
                cur = lr_min + 0.5 * (lr - lr_min) * (1.0 + math.cos(math.pi * it / total))
                self.net.step(lr=cur, wd=wd)
                it += 1
            hist.append(float(acc) / nb)
            if log and (ep % 10 == 0 or ep == epochs - 1):
                log(f"  epoch {ep} loss {hist[-1]:.4e}")
        return hist

    def predict(self, cases):
        """Standardised predictions (n, S, S, 5) as a float32 device tensor."""
        torch = self.torch
        n = len(cases)
        X = features(cases, self.S)
        out = torch.empty((n, self.S, self.S, NCH), dtype=torch.float32, device=self.net.dev)
        for j in range(0, n, self.B):
            chunk = X[j:j + self.B]
            k = chunk.shape[0]
            if k < self.B:
                chunk = np.concatenate([chunk, np.repeat(chunk[-1:], self.B - k, 0)])
            res = self.net.forward(torch.tensor(chunk, device=self.net.dev))
            out[j:j + k].copy_(res[:k])
        return out

    def affine(self, cfg: dict) -> list:
        """Map of the standardised channels to the fields mclbm_load_fields
        takes (u, v in lattice units, theta, phi, rho_f~ deviation)."""
        U, D = velocity_scale(cfg), density_scale(cfg)
        p0 = cfg["phi0"]
        s, m = self.std, self.mean
        return [U * s[0], U * s[1], s[2], p0 * s[3], D * s[4],
                U * m[0], U * m[1], m[2], p0 * (1.0 + m[3]), D * m[4]]

    def load(self, cavity, cfg: dict, pred) -> None:
        """Warm-start one cavity (or batch member) from its prediction."""
        cavity.load_fields(pred.contiguous(), affine=self.affine(cfg))

    def state(self) -> dict:
        st = {f"p_{k}": v for k, v in self.net.state().items()}
        st["mean"], st["std"] = self.mean, self.std
        return st

    def load_state(self, st: dict) -> None:
        self.net.load_state({k[2:]: v for k, v in st.items() if k.startswith("p_")})
        self.mean, self.std = np.asarray(st["mean"]), np.asarray(st["std"])


def run_to_steady(cases, warm: WarmStart | None = None, chunk: int = 500, tol: float = 1e-6,
                  max_steps: int = 4_000_000, drop: bool = True, log=None):
    """Run the cases as one batch from a cold start, or from the warm start
    ``warm``.  The solver's own criterion: the relative change of u and
    theta over ``chunk`` steps below ``tol``; with ``drop`` a cavity that
    meets it leaves the batch (and the run ends when all have), without it
    every cavity runs ``max_steps`` steps.  Records the hot-wall Nu and the
    residuals of every cavity after every chunk.  Returns a dict: steps
    (first chunk end meeting the criterion, 0 if none), converged, nu
    (final), times, walls (seconds of stepping at each record), nu_hist and
    res_hist (len(times) x n [x 2]), t_load (seconds of prediction and
    loading), seconds (of stepping), fields (final nondimensional fields)."""
    import time
    from . import Batch
    torch = warm.torch if warm is not None else __import__("torch")
    b = Batch([_cavity_kw(c) for c in cases])
    n = len(cases)
    t_load = 0.0
    if warm is not None:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pred = warm.predict(cases)
        for k, c in enumerate(cases):
            warm.load(b.members[k], c, pred[k])
        torch.cuda.synchronize()
        t_load = time.perf_counter() - t0
    steps = np.zeros(n, np.int64)
    alive = np.ones(n, bool)
    times, walls, hist, rhist = [], [], [], []
    b.residual(tol=0.0)
    t = 0
    t0 = time.perf_counter()
    while t < max_steps and alive.any():
        b.step(chunk)
        t += chunk
        res, st = b.residual(tol=tol if drop else 0.0)
        met = (res[:, 0] < tol) & (res[:, 1] < tol) & (st != 3)
        newly = met & (steps == 0)
        steps[newly] = t
        if drop:
            alive &= (st == 0)
        times.append(t)
        hist.append(b.nusselt()[:, 0].copy())
        rhist.append(res.copy())
        walls.append(time.perf_counter() - t0)
        if log and (t // chunk) % 200 == 0:
            log(f"  t={t} met the criterion {(steps > 0).sum()}/{n}")
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    fields = np.stack([nondimensional(b.members[k].moments(TARGETS), cases[k]) for k in range(n)])
    return dict(steps=steps, converged=steps > 0, nu=hist[-1], times=np.array(times),
                walls=np.array(walls), nu_hist=np.array(hist), res_hist=np.array(rhist), t_load=t_load,
                seconds=secs, fields=fields)


def run_mixed(cases, warm: WarmStart | None = None, storage: int = 1, switch_tol: float = 1e-4,
              chunk: int = 500, tol: float = 1e-6, max_steps: int = 4_000_000, log=None):
    """The transient with 16-bit population storage (``storage``: 1 FP16,
    2 BF16), the finish in FP32.  Every case starts (cold, or from ``warm``)
    in a 16-bit batch; when its change of u and theta over ``chunk`` steps
    falls below ``switch_tol`` it leaves that batch and its state moves to
    its member of an FP32 batch (``mclbm_copy_state``), which then runs it
    to the solver's own criterion (``tol``, drop-out).  Returns what
    ``run_to_steady`` returns, plus switched (the step of the move, 0 if
    none)."""
    import time
    from . import Batch
    torch = warm.torch if warm is not None else __import__("torch")
    n = len(cases)
    lo = Batch([dict(_cavity_kw(c), storage=storage) for c in cases])
    hi = Batch([_cavity_kw(c) for c in cases])
    t_load = 0.0
    if warm is not None:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pred = warm.predict(cases)
        for k, c in enumerate(cases):
            warm.load(lo.members[k], c, pred[k])
        torch.cuda.synchronize()
        t_load = time.perf_counter() - t0
    in_hi = np.zeros(n, bool)
    hi.set_active(in_hi.astype(np.int32))
    steps = np.zeros(n, np.int64)
    switched = np.zeros(n, np.int64)
    alive_lo = np.ones(n, bool)
    times, walls, hist, rhist = [], [], [], []
    lo.residual(tol=0.0)
    hi.residual(tol=0.0)
    t = 0
    t0 = time.perf_counter()
    while t < max_steps and (alive_lo.any() or (in_hi & (steps == 0)).any()):
        lo.step(chunk)
        hi.step(chunk)
        t += chunk
        res_lo, st_lo = lo.residual(tol=switch_tol)
        res_hi, st_hi = hi.residual(tol=tol)
        met = in_hi & (res_hi[:, 0] < tol) & (res_hi[:, 1] < tol) & (st_hi != 3)
        steps[met & (steps == 0)] = t
        # a moved cavity takes the 16-bit state and its residual reference
        # (the state now), so its next FP32 residual spans one chunk
        move = alive_lo & (st_lo == 1)
        alive_lo &= (st_lo == 0)
        for k in np.nonzero(move)[0]:
            hi.members[k].copy_state_from(lo.members[k])
            switched[k] = t
        if move.any():
            in_hi |= move
            hi.set_active((in_hi & (steps == 0)).astype(np.int32))
        nu = np.where(in_hi, hi.nusselt()[:, 0], lo.nusselt()[:, 0])
        times.append(t)
        hist.append(nu.copy())
        rhist.append(np.where(in_hi[:, None], res_hi, res_lo))
        walls.append(time.perf_counter() - t0)
        if log and (t // chunk) % 200 == 0:
            log(f"  t={t} switched {int((switched > 0).sum())}/{n}, met the criterion {(steps > 0).sum()}/{n}")
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    return dict(steps=steps, converged=steps > 0, switched=switched, nu=hist[-1], times=np.array(times),
                walls=np.array(walls), nu_hist=np.array(hist), res_hist=np.array(rhist), t_load=t_load,
                seconds=secs)


def run_plain(cases, chunk: int = 500, tol: float = 1e-6, max_steps: int = 4_000_000):
    """The plain way: every case alone, one after another, from a cold start
    in FP32 with one ``Cavity`` each, each until the solver's own criterion
    (as ``run_to_steady``).  Returns per case the records (steps, seconds
    since that case started, hot-wall Nu) and the steps and seconds at which
    the criterion was met (0 and the run's end if never)."""
    import time
    from . import Cavity
    out = []
    for c in cases:
        cav = Cavity(**_cavity_kw(c))
        cav.residual()
        t, rec = 0, []
        t0 = time.perf_counter()
        met = 0
        while t < max_steps:
            cav.step(chunk)
            t += chunk
            ru, rt = cav.residual()
            rec.append((t, time.perf_counter() - t0, cav.nusselt()[0]))
            if ru < tol and rt < tol:
                met = t
                break
        out.append(dict(records=np.array(rec), steps=met, seconds=rec[-1][1]))
        cav.close()
    return out


def settle_steps(times, nu_hist, nu_ref, rtol: float = 1e-3) -> np.ndarray:
    """Per cavity, the first recorded time from which on |Nu - Nu_ref| stays
    below rtol |Nu_ref| (the run's end if it never settles)."""
    out = np.zeros(nu_hist.shape[1], np.int64)
    for k in range(nu_hist.shape[1]):
        bad = np.nonzero(np.abs(nu_hist[:, k] - nu_ref[k]) > rtol * abs(nu_ref[k]))[0]
        if bad.size == 0:
            out[k] = times[0]
        elif bad[-1] + 1 < len(times):
            out[k] = times[bad[-1] + 1]
        else:
            out[k] = times[-1]
    return out


def main(argv=None) -> int:
    """Train a warm-start surrogate on solver steady states and compare the
    time to a steady hot-wall Nu (within 1e-3) from cold and warm starts on
    held-out cavities, possibly at a finer grid than the training one."""
    import argparse
    import json
    import time
    from . import inputs
    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--train-side", type=int, default=64)
    ap.add_argument("--train-count", type=int, default=256)
    ap.add_argument("--eval-side", type=int, default=128)
    ap.add_argument("--eval-count", type=int, default=16)
    ap.add_argument("--epochs", type=int, default=200)
    ap.add_argument("--channels", type=int, default=32)
    ap.add_argument("--modes", type=int, default=12)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--theta-weight", type=float, default=4.0)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--horizon", type=int, default=2_000_000, help="steps of both evaluation runs")
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--out", default=None)
    # A long evaluation can be split over several processes: train once and
    # save the model, then run the cold and the warm start separately (each
    # saving its run), then combine the two runs into the report.
    ap.add_argument("--save-model", default=None, help="write the trained model (.npz)")
    ap.add_argument("--load-model", default=None, help="skip data and training; use this model (.npz)")
    ap.add_argument("--eval", choices=("both", "cold", "warm", "none"), default="both")
    ap.add_argument("--save-run", default=None, help="write the evaluation run(s) made (.npz)")
    ap.add_argument("--combine", nargs=2, default=None, metavar=("COLD", "WARM"),
                    help="report from two saved runs instead of running")
    a = ap.parse_args(argv)
    import torch
    log = lambda s: print(s, flush=True)

    def cases(seed, n, side):
        return [dict(c, tau_f=-1.0) for c in inputs.sweep_parameters(seed, n, sides=(side,))]

    RUN_KEYS = ("steps", "converged", "nu", "times", "nu_hist", "seconds", "t_load", "fields")
    S = a.train_side
    train_rep = {"side": S}
    ws = None
    if a.combine:
        runs = [dict(np.load(f)) for f in a.combine]
        cold, warm = ({k: (r[k].item() if r[k].ndim == 0 else r[k]) for k in RUN_KEYS if k in r} for r in runs)
    else:
        if a.load_model:
            st = dict(np.load(a.load_model))
            S = int(st.pop("S"))
            C, m = int(st.pop("C")), int(st.pop("m"))
            train_rep = {k: (v.item() if v.ndim == 0 else v.tolist()) for k, v in st.items() if k.startswith("rep_")}
            train_rep = {k[4:]: v for k, v in train_rep.items()}
            ws = WarmStart(S=S, C=C, m=m, L=4, Q=64, B=a.batch, seed=a.seed)
            ws.load_state({k: v for k, v in st.items() if not k.startswith("rep_")})
            log(f"model loaded from {a.load_model} ({S}^2, C={C}, modes {m})")
        else:
            train = cases(a.seed * 1000 + 1, a.train_count, S)
            t0 = time.perf_counter()
            F, steps, ok = generate_dataset(train, chunk=2000, tol=a.tol, max_steps=2_000_000, log=log)
            torch.cuda.synchronize()
            t_gen = time.perf_counter() - t0
            log(f"training data: {ok.sum()}/{len(train)} cavities of {S}^2 converged in {t_gen:.1f} s")
            ws = WarmStart(S=S, C=a.channels, m=min(a.modes, S // 4), L=4, Q=64, B=a.batch, seed=a.seed)
            t0 = time.perf_counter()
            hist = ws.fit([c for c, o in zip(train, ok) if o], F[ok], epochs=a.epochs, lr=a.lr,
                          weights=(1, 1, a.theta_weight, 1, 1),
                          log=lambda s: log(s) if s.strip().startswith("epoch") else None)
            torch.cuda.synchronize()
            t_train = time.perf_counter() - t0
            log(f"trained {a.epochs} epochs in {t_train:.1f} s, loss {hist[0]:.3e} -> {hist[-1]:.3e}")
            train_rep = {"side": S, "count": int(ok.sum()), "epochs": a.epochs, "channels": a.channels,
                         "modes": min(a.modes, S // 4), "seconds_data": t_gen, "seconds_train": t_train,
                         "loss_first": hist[0], "loss_last": hist[-1]}
            if a.save_model:
                np.savez(a.save_model, S=S, C=a.channels, m=min(a.modes, S // 4), **ws.state(),
                         **{"rep_" + k: v for k, v in train_rep.items()})
        test = cases(a.seed * 1000 + 2, a.eval_count, a.eval_side)
        # Both starts run the same fixed horizon without drop-out, so that
        # the steady Nu is taken well past the stopping criterion (which
        # leaves a drift of order tol times the slowest decay time over the
        # chunk) and the two final states can be compared.
        cold = warm = None
        if a.eval in ("both", "cold"):
            cold = run_to_steady(test, None, chunk=500, tol=a.tol, max_steps=a.horizon, drop=False, log=log)
            log(f"cold start: {cold['converged'].sum()}/{len(test)} met the criterion, {cold['seconds']:.1f} s")
        if a.eval in ("both", "warm"):
            warm = run_to_steady(test, ws, chunk=500, tol=a.tol, max_steps=a.horizon, drop=False, log=log)
            log(f"warm start: {warm['converged'].sum()}/{len(test)} met the criterion, {warm['seconds']:.1f} s "
                f"(prediction and loading {warm['t_load'] * 1e3:.1f} ms)")
        if a.save_run:
            made = cold if cold is not None else warm
            if made is not None:
                # the final fields only serve an evaluation at the training
                # resolution; large evaluations leave them out of the file
                keep = [k for k in RUN_KEYS if k != "fields" or np.asarray(made[k]).nbytes <= (32 << 20)]
                np.savez(a.save_run, **{k: np.asarray(made[k]) for k in keep})
        if cold is None or warm is None:
            return 0
    done = cold["converged"] & warm["converged"]
    nu_inf = cold["nu"]
    sc = settle_steps(cold["times"], cold["nu_hist"], nu_inf)
    sw = settle_steps(warm["times"], warm["nu_hist"], nu_inf)
    dnu = np.abs(warm["nu"] - nu_inf) / np.abs(nu_inf)
    per_step = cold["seconds"] / cold["times"][-1]
    rep = {
        "train": train_rep,
        "eval": {"side": a.eval_side, "count": len(cold["nu"]), "tol": a.tol, "horizon": a.horizon,
                 "cold_settle_steps": sc.tolist(), "warm_settle_steps": sw.tolist(),
                 "settle_ratio_total": float(sc.sum() / max(sw.sum(), 1)),
                 "settle_ratio_median": float(np.median(sc / np.maximum(sw, 1))),
                 "cold_criterion_steps": cold["steps"].tolist(), "warm_criterion_steps": warm["steps"].tolist(),
                 "criterion_ratio_total": float(cold["steps"][done].sum() / max(warm["steps"][done].sum(), 1)),
                 "met_both": int(done.sum()),
                 "final_nu_rel_diff_max": float(dnu.max()),
                 "seconds_per_batch_step": per_step,
                 "seconds_to_settle_cold": float(sc.max() * per_step),
                 "seconds_to_settle_warm": float(sw.max() * per_step + warm["t_load"]),
                 "seconds_load": warm["t_load"]},
    }
    if a.eval_side == S and ws is not None and "fields" in cold:
        pred = ws.predict(test).cpu().numpy() * ws.std + ws.mean
        err = np.sqrt(((pred - cold["fields"]) ** 2).reshape(-1, NCH).mean(0)) / cold["fields"].reshape(-1, NCH).std(0)
        rep["eval"]["rel_rms_error"] = dict(zip(("u", "v", "theta", "phi", "rho_f"), err.tolist()))
    log(json.dumps(rep["eval"]))
    if a.out:
        with open(a.out, "w") as fh:
            json.dump(rep, fh, indent=1)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
