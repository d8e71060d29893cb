"""Surrogate kernels on the GPU: the BF16 matrix-core GEMM against FP64
products of the BF16-rounded operands, the elementwise kernels against their
definitions, and the whole network (forward pass and every gradient) against
the FP64 autograd oracle."""
import ctypes
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from oracle import fno_oracle  # noqa: E402
import paper_1511_04552_amd as mc  # noqa: E402
from paper_1511_04552_amd import surrogate  # noqa: E402

DEV = torch.device("cuda")


def bf16(a: np.ndarray) -> np.ndarray:
    """Round float32 to the nearest bfloat16 (ties to even), as float64."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def _gemm(ta, tb, M, N, K, alpha, A, lda, sa, B, ldb, sb, beta, C, ldc, sc, nb1, nb2):
    s = torch.cuda.current_stream()
    rc = mc.lib().mclbm_nn_gemm(ta, tb, M, N, K, alpha, ctypes.c_void_p(A.data_ptr()), lda, sa[0], sa[1],
                                ctypes.c_void_p(B.data_ptr()), ldb, sb[0], sb[1], beta,
                                ctypes.c_void_p(C.data_ptr()), ldc, sc[0], sc[1], nb1, nb2,
                                ctypes.c_void_p(s.cuda_stream))
    assert rc == 0, mc.lib().mclbm_last_error()
    torch.cuda.synchronize()


@pytest.mark.parametrize("ta,tb", [(0, 0), (0, 1), (1, 0), (1, 1)])
@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (70, 33, 45), (130, 65, 97), (16, 64, 300)])
def test_gemm_matches_fp64_of_bf16_operands(ta, tb, M, N, K):
    """Ragged sizes over several 64 x 64 x 32 tiles, both transposes,
    alpha/beta, two-level batch strides with padding in the leading
    dimensions."""
    rng = np.random.default_rng(M * 1000 + N * 10 + K + 7 * ta + 3 * tb)
    nb1, nb2 = 2, 3
    ar, ac = (K, M) if ta else (M, K)
    br, bc = (N, K) if tb else (K, N)
    lda, ldb, ldc = ac + 3, bc + 1, N + 5
    sa2, sb2, sc2 = ar * lda + 7, br * ldb, M * ldc + 2
    sa1, sb1, sc1 = nb2 * sa2 + 11, 0, nb2 * sc2        # B broadcast over z1
    A = rng.normal(size=nb1 * sa1).astype(np.float32)
    B = rng.normal(size=nb2 * sb2 + 5).astype(np.float32)
    C0 = rng.normal(size=nb1 * sc1 + 9).astype(np.float32)
    alpha, beta = 0.75, -0.5
    tA, tB, tC = (torch.tensor(x, device=DEV) for x in (A, B, C0))
    _gemm(ta, tb, M, N, K, alpha, tA, lda, (sa1, sa2), tB, ldb, (sb1, sb2), beta, tC, ldc, (sc1, sc2), nb1, nb2)
    got = tC.cpu().numpy().astype(np.float64)
    Ab, Bb = bf16(A), bf16(B)
    ref = C0.astype(np.float64).copy()
    for z1 in range(nb1):
        for z2 in range(nb2):
            a = Ab[z1 * sa1 + z2 * sa2:][:ar * lda].reshape(ar, lda)[:, :ac]
            b = Bb[z1 * sb1 + z2 * sb2:][:br * ldb].reshape(br, ldb)[:, :bc]
            opa = a.T if ta else a
            opb = b.T if tb else b
            o = z1 * sc1 + z2 * sc2
            cv = ref[o:o + M * ldc].reshape(M, ldc)
            absprod = np.abs(opa) @ np.abs(opb)
            cv[:, :N] = alpha * (opa @ opb) + beta * cv[:, :N]
            g = got[o:o + M * ldc].reshape(M, ldc)[:, :N]
            # FP32 accumulation of exact BF16 products: K roundings at most
            bound = 2.0 * K * 2.0 ** -24 * abs(alpha) * absprod + 2.0 ** -23 * np.abs(cv[:, :N]) + 1e-30
            assert (np.abs(g - cv[:, :N]) <= bound).all(), (z1, z2, np.abs(g - cv[:, :N]).max())
    # elements outside the M x N windows are untouched
    mask = np.ones_like(ref, dtype=bool)
    for z1 in range(nb1):
        for z2 in range(nb2):
            o = z1 * sc1 + z2 * sc2
            for r in range(M):
                mask[o + r * ldc:o + r * ldc + N] = False
    assert np.array_equal(got[mask], C0.astype(np.float64)[mask])


@pytest.mark.parametrize("tb", [0, 1])
@pytest.mark.parametrize("M,N,K", [(128, 256, 32), (256, 512, 160), (384, 256, 64)])
def test_large_tile_gemm_matches_fp64_of_bf16_operands(tb, M, N, K):
    """Shapes that take the 128 x 256 large-tile kernel (M % 128, N % 256,
    K % 32, 16-byte aligned rows and batch offsets), with both layouts of B,
    two-level batches, padded leading dimensions and alpha/beta: the same
    bound as the general kernel."""
    rng = np.random.default_rng(M + N + K + tb)
    nb1, nb2 = 2, 2
    br, bc = (N, K) if tb else (K, N)
    lda, ldb, ldc = K + 4, bc + 8, N + 3
    sa2, sb2, sc2 = M * lda + 4, br * ldb + 12, M * ldc + 1
    sa1, sb1, sc1 = nb2 * sa2 + 8, nb2 * sb2, nb2 * sc2
    A = rng.normal(size=nb1 * sa1).astype(np.float32)
    B = rng.normal(size=nb1 * sb1).astype(np.float32)
    C0 = rng.normal(size=nb1 * sc1).astype(np.float32)
    alpha, beta = 1.25, 0.5
    tA, tB, tC = (torch.tensor(x, device=DEV) for x in (A, B, C0))
    _gemm(0, tb, M, N, K, alpha, tA, lda, (sa1, sa2), tB, ldb, (sb1, sb2), beta, tC, ldc, (sc1, sc2), nb1, nb2)
    got = tC.cpu().numpy().astype(np.float64)
    Ab, Bb = bf16(A), bf16(B)
    for z1 in range(nb1):
        for z2 in range(nb2):
            a = Ab[z1 * sa1 + z2 * sa2:][:M * lda].reshape(M, lda)[:, :K]
            b = Bb[z1 * sb1 + z2 * sb2:][:br * ldb].reshape(br, ldb)[:, :bc]
            opb = b.T if tb else b
            o = z1 * sc1 + z2 * sc2
            c0 = C0[o:o + M * ldc].astype(np.float64).reshape(M, ldc)[:, :N]
            ref = alpha * (a @ opb) + beta * c0
            bound = 2.0 * K * 2.0 ** -24 * abs(alpha) * (np.abs(a) @ np.abs(opb)) + 2.0 ** -23 * np.abs(ref) + 1e-30
            g = got[o:o + M * ldc].reshape(M, ldc)[:, :N]
            assert (np.abs(g - ref) <= bound).all(), (z1, z2, np.abs(g - ref).max())


def test_large_gemm_sampled_rows_2048():
    """2048^3 with the large-tile kernel: sampled rows of C (every tile row
    position, both wave halves) against FP64 products of the BF16-rounded
    operands."""
    n = 2048
    g = torch.Generator(device="cpu").manual_seed(5)
    A = torch.randn(n, n, generator=g)
    B = torch.randn(n, n, generator=g)
    tA, tB = A.to(DEV), B.to(DEV)
    tC = torch.zeros(n, n, device=DEV)
    _gemm(0, 0, n, n, n, 1.0, tA, n, (0, 0), tB, n, (0, 0), 0.0, tC, n, (0, 0), 1, 1)
    rows = np.array([0, 1, 31, 32, 63, 64, 100, 127, 128, 1000, 2047])
    Ab, Bb = bf16(A.numpy()), bf16(B.numpy())
    ref = Ab[rows] @ Bb
    bound = 2.0 * n * 2.0 ** -24 * (np.abs(Ab[rows]) @ np.abs(Bb)) + 1e-30
    got = tC.cpu().numpy()[rows].astype(np.float64)
    assert (np.abs(got - ref) <= bound).all(), np.abs(got - ref).max()


@pytest.mark.parametrize("tb", [0, 1])
def test_large_tile_gemm_many_batches_matches_fp64_of_bf16_operands(tb):
    """16 products of 1024 x 1024 x 96 through the large-tile kernel (512
    tiles over the batch), padded leading dimensions, two-level batch
    offsets and alpha/beta: every element within the bound of the general
    kernel, and nothing written outside the products."""
    M = N = 1024
    K = 96
    rng = np.random.default_rng(17 + tb)
    nb1, nb2 = 4, 4
    br, bc = (N, K) if tb else (K, N)
    lda, ldb, ldc = K + 4, bc + 4, N + 1
    sa2, sb2, sc2 = M * lda + 4, br * ldb + 4, M * ldc
    sa1, sb1, sc1 = nb2 * sa2, nb2 * sb2 + 8, nb2 * sc2 + 3
    A = rng.normal(size=nb1 * sa1).astype(np.float32)
    B = rng.normal(size=nb1 * sb1).astype(np.float32)
    C0 = rng.normal(size=nb1 * sc1).astype(np.float32)
    alpha, beta = 0.75, -0.5
    tA, tB, tC = (torch.tensor(x, device=DEV) for x in (A, B, C0))
    _gemm(0, tb, M, N, K, alpha, tA, lda, (sa1, sa2), tB, ldb, (sb1, sb2), beta, tC, ldc, (sc1, sc2), nb1, nb2)
    got = tC.cpu().numpy().astype(np.float64)
    Ab, Bb = bf16(A), bf16(B)
    for z1 in range(nb1):
        for z2 in range(nb2):
            a = Ab[z1 * sa1 + z2 * sa2:][:M * lda].reshape(M, lda)[:, :K]
            b = Bb[z1 * sb1 + z2 * sb2:][:br * ldb].reshape(br, ldb)[:, :bc]
            opb = b.T if tb else b
            o = z1 * sc1 + z2 * sc2
            c0 = C0[o:o + M * ldc].astype(np.float64).reshape(M, ldc)[:, :N]
            ref = alpha * (a @ opb) + beta * c0
            bound = 2.0 * K * 2.0 ** -24 * abs(alpha) * (np.abs(a) @ np.abs(opb)) + 2.0 ** -23 * np.abs(ref) + 1e-30
            g = got[o:o + M * ldc].reshape(M, ldc)[:, :N]
            assert (np.abs(g - ref) <= bound).all(), (z1, z2, np.abs(g - ref).max())
    # the C elements outside the products are untouched
    mask = np.ones(nb1 * sc1, bool)
    for z1 in range(nb1):
        for z2 in range(nb2):
            o = z1 * sc1 + z2 * sc2
            mask[o:o + M * ldc].reshape(M, ldc)[:, :N] = False
    assert np.array_equal(got[mask], C0.astype(np.float64)[mask])


@pytest.mark.parametrize("tb", [0, 1])
def test_large_gemm_sampled_rows_4096(tb):
    """4096^3, the benchmarked product, with both layouts of B: sampled rows
    of C (every row position of a wave's block and the tile edges) against
    FP64 products of the BF16-rounded operands."""
    n = 4096
    g = torch.Generator(device="cpu").manual_seed(7 + tb)
    A = torch.randn(n, n, generator=g)
    B = torch.randn(n, n, generator=g)
    tA, tB = A.to(DEV), B.to(DEV)
    tC = torch.zeros(n, n, device=DEV)
    _gemm(0, tb, n, n, n, 1.0, tA, n, (0, 0), tB, n, (0, 0), 0.0, tC, n, (0, 0), 1, 1)
    rows = np.array([0, 1, 31, 32, 63, 64, 127, 128, 191, 192, 255, 256, 2100, 4095])
    Ab, Bb = bf16(A.numpy()), bf16(B.numpy())
    opb = Bb.T if tb else Bb
    ref = Ab[rows] @ opb
    bound = 2.0 * n * 2.0 ** -24 * (np.abs(Ab[rows]) @ np.abs(opb)) + 1e-30
    got = tC.cpu().numpy()[rows].astype(np.float64)
    assert (np.abs(got - ref) <= bound).all(), np.abs(got - ref).max()


def test_gemm_beta_zero_ignores_nan_in_c():
    A = torch.ones(4, 4, device=DEV)
    C = torch.full((4, 4), float("nan"), device=DEV)
    _gemm(0, 0, 4, 4, 4, 1.0, A, 4, (0, 0), A, 4, (0, 0), 0.0, C, 4, (0, 0), 1, 1)
    assert torch.equal(C, torch.full((4, 4), 4.0, device=DEV))


def test_gemm_rejects_bad_arguments():
    L = mc.lib()
    A = torch.ones(4, 4, device=DEV)
    p = ctypes.c_void_p(A.data_ptr())
    assert L.mclbm_nn_gemm(0, 0, 0, 4, 4, 1.0, p, 4, 0, 0, p, 4, 0, 0, 0.0, p, 4, 0, 0, 1, 1, None) == mc.EINVAL
    assert L.mclbm_nn_gemm(0, 0, 4, 4, 4, 1.0, p, 3, 0, 0, p, 4, 0, 0, 0.0, p, 4, 0, 0, 1, 1, None) == mc.EINVAL
    assert L.mclbm_nn_gemm(0, 0, 4, 4, 4, 1.0, None, 4, 0, 0, p, 4, 0, 0, 0.0, p, 4, 0, 0, 1, 1, None) == mc.EINVAL


def _phi(x):
    return 0.5 * (1.0 + np.vectorize(math.erf)(x / math.sqrt(2.0)))


def test_elementwise_kernels_match_definitions():
    rng = np.random.default_rng(3)
    ops = surrogate._Ops(torch, torch.cuda.current_stream())
    rows, cols = 1037, 70
    y0 = rng.normal(size=(rows, cols)).astype(np.float32) * 3
    bias = rng.normal(size=cols).astype(np.float32)
    y, pre = torch.tensor(y0, device=DEV), torch.zeros(rows, cols, device=DEV)
    ops.bias_act(y, torch.tensor(bias, device=DEV), rows, cols, surrogate.GELU, pre)
    x = y0.astype(np.float64) + bias
    np.testing.assert_allclose(pre.cpu().numpy(), x, rtol=1e-6, atol=1e-6)
    np.testing.assert_allclose(y.cpu().numpy(), x * _phi(x), rtol=2e-6, atol=2e-6)
    # identity, no bias
    y2 = torch.tensor(y0, device=DEV)
    ops.bias_act(y2, None, rows, cols, surrogate.IDENT)
    assert torch.equal(y2, torch.tensor(y0, device=DEV))
    # GELU derivative
    dy0 = rng.normal(size=(rows, cols)).astype(np.float32)
    dy = torch.tensor(dy0, device=DEV)
    ops.act_backward(dy, pre, surrogate.GELU)
    dgelu = _phi(x) + x * np.exp(-0.5 * x * x) / math.sqrt(2 * math.pi)
    np.testing.assert_allclose(dy.cpu().numpy(), dy0 * dgelu, rtol=2e-5, atol=2e-6)
    # column sums
    scratch = torch.zeros(int(mc.lib().mclbm_nn_colsum_scratch(rows, cols)), device=DEV)
    db = torch.full((cols,), 2.0, device=DEV)
    ops.colsum(torch.tensor(y0, device=DEV), db, rows, cols, scratch, beta=0.5)
    np.testing.assert_allclose(db.cpu().numpy(), 1.0 + y0.astype(np.float64).sum(0), rtol=1e-5, atol=1e-4)
    # mean-squared error
    n = 12345
    a = rng.normal(size=n).astype(np.float32)
    t = rng.normal(size=n).astype(np.float32)
    d = torch.zeros(n, device=DEV)
    ms = torch.zeros(int(mc.lib().mclbm_nn_mse_scratch(n)), dtype=torch.float64, device=DEV)
    loss = torch.zeros(1, dtype=torch.float64, device=DEV)
    ops.mse(torch.tensor(a, device=DEV), torch.tensor(t, device=DEV), d, ms, loss)
    # the residual y - t is formed in FP32, its square summed in FP64
    diff = (a - t).astype(np.float64)
    assert abs(float(loss) - (diff ** 2).mean()) <= 1e-12 * (diff ** 2).mean()
    np.testing.assert_allclose(d.cpu().numpy(), 2 * diff / n, rtol=1e-6)


def test_adamw_matches_update_rule():
    rng = np.random.default_rng(4)
    n = 3001
    w0, m0 = rng.normal(size=n), 0.1 * rng.normal(size=n)
    v0 = rng.uniform(0, 1, n)
    g0 = rng.normal(size=n)
    tw, tg, tm, tv = (torch.tensor(x.astype(np.float32), device=DEV) for x in (w0, g0, m0, v0))
    ops = surrogate._Ops(torch, torch.cuda.current_stream())
    lr, b1, b2, eps, wd, t = 1e-2, 0.9, 0.99, 1e-8, 1e-3, 5
    ops.adamw(tw, tg, tm, tv, lr, b1, b2, eps, wd, t)
    w32, g32, m32, v32 = (x.astype(np.float32).astype(np.float64) for x in (w0, g0, m0, v0))
    m = b1 * m32 + (1 - b1) * g32
    v = b2 * v32 + (1 - b2) * g32 ** 2
    w = w32 - lr * (m / (1 - b1 ** t) / (np.sqrt(v / (1 - b2 ** t)) + eps) + wd * w32)
    np.testing.assert_allclose(tm.cpu().numpy(), m, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(tv.cpu().numpy(), v, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(tw.cpu().numpy(), w, rtol=1e-5, atol=1e-6)


# ------------------------------------------------------------ the network ---

def _relerr(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-30))


@pytest.mark.parametrize("S,C,m,L,Q,B", [(16, 8, 4, 2, 16, 2), (24, 12, 5, 3, 20, 3)])
def test_network_forward_and_gradients_match_fp64_oracle(S, C, m, L, Q, B):
    """Forward pass and the gradient of every parameter against FP64 autograd.
    The GPU rounds every GEMM operand to BF16 (unit roundoff 2^-9 = 2e-3);
    through a dozen chained products the normwise relative error stays
    within 3e-2, which is the bound used here."""
    net = surrogate.FNO(S=S, C=C, m=m, L=L, Q=Q, B=B, seed=11)
    rng = np.random.default_rng(12)
    # larger random spectral weights than the initialisation so that the
    # spectral path carries weight in the check
    for l in range(L):
        for k in (f"R_re_{l}", f"R_im_{l}"):
            net.params[k].copy_(torch.tensor(rng.normal(0, 0.5 / C, net.params[k].shape).astype(np.float32)))
    for k in ("b_lift", "c1", "c2") + tuple(f"b_{l}" for l in range(L)):
        net.params[k].copy_(torch.tensor(rng.normal(0, 0.1, net.params[k].shape).astype(np.float32)))
    a = rng.normal(size=(B, S, S, 5)).astype(np.float32)
    t = rng.normal(size=(B, S, S, 5)).astype(np.float32)
    out = net.forward(torch.tensor(a, device=DEV))
    loss = net.backward(torch.tensor(t, device=DEV))
    torch.cuda.synchronize()
    p64 = {k: torch.tensor(v.cpu().numpy().astype(np.float64)) for k, v in net.params.items()}
    ref_out, ref_loss, ref_g = fno_oracle.loss_and_grads(p64, torch.tensor(a, dtype=torch.float64),
                                                        torch.tensor(t, dtype=torch.float64), m)
    assert _relerr(out.cpu().numpy(), ref_out.numpy()) < 3e-2
    assert abs(float(loss) - ref_loss) < 3e-2 * ref_loss
    for k, g in ref_g.items():
        e = _relerr(net.grads[k].cpu().numpy(), g.numpy())
        assert e < 3e-2, (k, e)


def test_training_reduces_loss():
    """Fitting a fixed smooth target: AdamW steps through the kernels reduce
    the loss by an order of magnitude."""
    S, B = 16, 4
    net = surrogate.FNO(S=S, C=16, m=4, L=2, Q=32, B=B, seed=3, nout=4)
    rng = np.random.default_rng(5)
    xs = (np.arange(S) + 0.5) / S
    a = np.zeros((B, S, S, 5), np.float32)
    t = np.zeros((B, S, S, 4), np.float32)
    for b in range(B):
        p = rng.uniform(-1, 1, 3)
        a[b, :, :, :3] = p
        a[b, :, :, 3] = xs[None, :]
        a[b, :, :, 4] = xs[:, None]
        t[b, :, :, 0] = p[0] * np.sin(np.pi * xs[None, :]) * np.cos(np.pi * xs[:, None])
        t[b, :, :, 2] = 0.5 - xs[None, :] + 0.2 * p[1] * np.sin(2 * np.pi * xs[:, None])
        t[b, :, :, 3] = p[2] * xs[:, None]
    ta, tt = torch.tensor(a, device=DEV), torch.tensor(t, device=DEV)
    losses = []
    for it in range(300):
        net.forward(ta)
        losses.append(float(net.backward(tt)))
        net.step(lr=3e-3)
    assert np.isfinite(losses).all()
    assert losses[-1] < 0.1 * losses[0], (losses[0], losses[-1])
