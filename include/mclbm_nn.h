/*
 * mclbm_nn.h -- C ABI of the dense kernels of the warm-start surrogate.
 *
 * The surrogate maps the cavity parameters (Ra, phi0, d_p) and a coordinate
 * grid to near-steady fields (u, v, theta, phi); the lattice Boltzmann solver
 * then starts from those fields (mclbm_load_fields in mclbm.h) and still
 * runs to its own convergence criterion, so the surrogate changes only the
 * time to steady state, never the converged answer.  Its network is a
 * Fourier neural operator whose spectral layers are discrete Fourier
 * transforms written as matrix products; every matrix product runs on the
 * BF16 matrix cores of gfx950 with FP32 accumulation (mclbm_nn_gemm), and
 * training uses the elementwise kernels below.
 *
 * Conventions as in mclbm.h: int status returns (MCLBM_OK = 0), device
 * pointers, work enqueued on `stream`, async unless noted, no allocation.
 * All matrices are row-major FP32 in memory; the GEMM rounds its operands to
 * BF16 (round to nearest even) when it stages them and accumulates in FP32.
 */
#ifndef MCLBM_NN_H
#define MCLBM_NN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Strided batched GEMM:  C_z = alpha * op(A_z) op(B_z) + beta * C_z  for
 * z = z1 * nb2 + z2, z1 < nb1, z2 < nb2, with
 *   A_z = A + z1*sa1 + z2*sa2 (elements), likewise B_z, C_z.
 * op(A) is M x K: ta == 0 -> A is M x K (row stride lda >= K);
 *                 ta == 1 -> A is K x M (row stride lda >= M).
 * op(B) is K x N: tb == 0 -> B is K x N (ldb >= N); tb == 1 -> N x K (ldb >= K).
 * C is M x N with row stride ldc >= N.  beta == 0 does not read C.
 * Strides may be 0 (broadcast).  M, N, K >= 1, nb1, nb2 >= 1,
 * nb1 * nb2 <= 65535 and ceil(M / 64) <= 65535 (MCLBM_EINVAL otherwise).
 * Products with ta == 0, M % 128 == 0, N % 256 == 0, K % 32 == 0, leading
 * dimensions and batch strides of A and B multiples of 4, A and B 16-byte
 * aligned and each batch entry's operands within 2^31 bytes run on a
 * large-tile kernel (128 x 256 tiles of C, 32 x 32 x 16 MFMAs); all others
 * on a general 64 x 64 kernel.  Both round the operands identically; the
 * order of the FP32 accumulation differs. */
int mclbm_nn_gemm(int32_t ta, int32_t tb, int32_t M, int32_t N, int32_t K, float alpha,
                  const float* A, int64_t lda, int64_t sa1, int64_t sa2,
                  const float* B, int64_t ldb, int64_t sb1, int64_t sb2,
                  float beta, float* C, int64_t ldc, int64_t sc1, int64_t sc2,
                  int32_t nb1, int32_t nb2, void* stream);

/* Activations: 0 = identity, 1 = GELU (x/2 (1 + erf(x/sqrt 2))). */
enum { MCLBM_NN_ID = 0, MCLBM_NN_GELU = 1 };

/* y[r, c] = act(y[r, c] + bias[c]) over rows x cols (bias may be NULL);
 * if pre != NULL it receives the argument of act (for the backward pass). */
int mclbm_nn_bias_act(float* y, const float* bias, int64_t rows, int32_t cols, int32_t act,
                      float* pre, void* stream);

/* dy[k] *= act'(pre[k]) for k < n. */
int mclbm_nn_act_backward(float* dy, const float* pre, int64_t n, int32_t act, void* stream);

/* db[c] = beta * db[c] + sum_r dy[r, c]: column sums in a fixed order
 * through the caller's scratch of mclbm_nn_colsum_scratch(rows, cols)
 * floats. */
int64_t mclbm_nn_colsum_scratch(int64_t rows, int32_t cols);
int mclbm_nn_colsum(const float* dy, float* db, int64_t rows, int32_t cols, float beta,
                    float* scratch, void* stream);

/* Mean-squared error: dy[k] = 2 (y[k] - t[k]) / n and
 * loss_out[0] = sum (y - t)^2 / n (FP64, fixed-order reduction through the
 * caller's scratch of mclbm_nn_mse_scratch(n) doubles). */
int64_t mclbm_nn_mse_scratch(int64_t n);
int mclbm_nn_mse(const float* y, const float* t, float* dy, int64_t n, double* scratch,
                 double* loss_out, void* stream);

/* AdamW step t >= 1 (bias-corrected, decoupled weight decay):
 * m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 * w -= lr (m / (1-b1^t) / (sqrt(v / (1-b2^t)) + eps) + wd w). */
int mclbm_nn_adamw(float* w, const float* g, float* m, float* v, int64_t n, float lr,
                   float b1, float b2, float eps, float wd, int32_t t, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* MCLBM_NN_H */
