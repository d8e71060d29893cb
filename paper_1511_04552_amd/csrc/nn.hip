// Dense kernels of the warm-start surrogate (C ABI in include/mclbm_nn.h):
// a strided-batched GEMM on the BF16 matrix cores of gfx950 with FP32
// accumulation, and the elementwise kernels of training.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>

#include "mclbm.h"
#include "mclbm_nn.h"

namespace mclbm_host {
void set_last_error(const std::string& msg);  // the library's thread-local message
}

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

struct GemmArgs {
  int ta, tb, M, N, K, nb2;
  float alpha, beta;
  const float* A;
  long long lda, sa1, sa2;
  const float* B;
  long long ldb, sb1, sb2;
  float* C;
  long long ldc, sc1, sc2;
};

constexpr int BM = 64, BN = 64, BK = 32;
constexpr int LDK = BK + 8;  // padded row of the LDS tiles (80 bytes: 16-byte aligned)

// One 64 x 64 tile of C per 256-thread workgroup.  The four waves own
// 32 x 32 quadrants, each four 16 x 16 x 32 BF16 MFMAs per K step.  Operand
// tiles are staged through LDS as [row][k] (A) and [col][k] (B), so every
// lane reads its eight consecutive K values of one row / column with one
// 16-byte LDS load: lane l holds row (l mod 16), K values 8 (l div 16) .. +7;
// the 4 accumulators of lane l are column (l mod 16), rows 4 (l div 16) + r.
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
  __shared__ __attribute__((aligned(16))) __bf16 As[BM][LDK];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[BN][LDK];
  const long long z = blockIdx.z;
  const long long z1 = z / g.nb2, z2 = z % g.nb2;
  const float* __restrict__ A = g.A + z1 * g.sa1 + z2 * g.sa2;
  const float* __restrict__ B = g.B + z1 * g.sb1 + z2 * g.sb2;
  float* __restrict__ C = g.C + z1 * g.sc1 + z2 * g.sc2;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  f32x4 acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  for (int k0 = 0; k0 < g.K; k0 += BK) {
    // stage A (M x K view), coalesced along the contiguous index
    for (int e = tid; e < BM * BK; e += 256) {
      int r, kk;
      if (g.ta == 0) { r = e / BK; kk = e % BK; } else { r = e % BM; kk = e / BM; }
      const int m = m0 + r, k = k0 + kk;
      float v = 0.f;
      if (m < g.M && k < g.K) v = g.ta == 0 ? A[(long long)m * g.lda + k] : A[(long long)k * g.lda + m];
      As[r][kk] = (__bf16)v;
    }
    // stage B (K x N view) as [n][k]
    for (int e = tid; e < BN * BK; e += 256) {
      int c, kk;
      if (g.tb == 0) { c = e % BN; kk = e / BN; } else { c = e / BK; kk = e % BK; }
      const int n = n0 + c, k = k0 + kk;
      float v = 0.f;
      if (n < g.N && k < g.K) v = g.tb == 0 ? B[(long long)k * g.ldb + n] : B[(long long)n * g.ldb + k];
      Bs[c][kk] = (__bf16)v;
    }
    __syncthreads();
    const int kq = 8 * (lane >> 4), rl = lane & 15;
    bf16x8 a[2], b[2];
    for (int i = 0; i < 2; ++i) a[i] = *reinterpret_cast<const bf16x8*>(&As[wm + 16 * i + rl][kq]);
    for (int j = 0; j < 2; ++j) b[j] = *reinterpret_cast<const bf16x8*>(&Bs[wn + 16 * j + rl][kq]);
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    __syncthreads();
  }
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm + 16 * i + 4 * (lane >> 4) + r;
        const int n = n0 + wn + 16 * j + (lane & 15);
        if (m < g.M && n < g.N) {
          float* c = C + (long long)m * g.ldc + n;
          const float v = g.alpha * acc[i][j][r];
          *c = g.beta == 0.f ? v : v + g.beta * *c;
        }
      }
}

// Large products: C tiles of 128 x 256 per 256-thread workgroup, op(A) = A
// (M x K row-major), op(B) = B (K x N, TB = 0) or B^T (B is N x K, TB = 1),
// M % 128 == 0, N % 256 == 0, K % 32 == 0, every row and batch offset
// 16-byte aligned (checked by the host).  The four waves own 64 x 128
// quadrants: per 16-wide K step each runs 2 x 4 MFMAs of 32 x 32 x 16
// (FP32 accumulation).  The operands of the next 32-wide K step are loaded
// into registers (16-byte loads) while the
// current step computes, then rounded to BF16 and written to LDS as
// [row][k] (a K x N B is read as 16-byte row pieces and transposed in
// registers), so that each MFMA operand is one 16-byte LDS read: lane l holds
// row (l mod 32), K values 8 (l div 32) .. +7.  Accumulator r of lane l is
// row 8 (r div 4) + 4 (l div 32) + (r mod 4), column (l mod 32).
typedef float f32x16 __attribute__((ext_vector_type(16)));
constexpr int GM = 128, GN = 256, GK = 32, GLK = GK + 8;

__device__ __forceinline__ unsigned gemm_tile(unsigned b, unsigned nb) {
  // workgroups are dealt round-robin to the 8 XCDs: give each XCD one
  // contiguous run of tiles (row-major over the C tiles), so that the A row
  // panels and B column panels it reads stay in its own L2
  const unsigned q = nb >> 3, r = nb & 7u, k = b & 7u;
  return k * q + (k < r ? k : r) + (b >> 3);
}

template <int TB>
__global__ __launch_bounds__(256, 2) void k_gemm_big(GemmArgs g) {
  __shared__ __attribute__((aligned(16))) __bf16 As[GM][GLK];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[GN][GLK];
  const long long z = blockIdx.z;
  const long long z1 = z / g.nb2, z2 = z % g.nb2;
  const float* __restrict__ A = g.A + z1 * g.sa1 + z2 * g.sa2;
  const float* __restrict__ B = g.B + z1 * g.sb1 + z2 * g.sb2;
  float* __restrict__ C = g.C + z1 * g.sc1 + z2 * g.sc2;
  const unsigned tiles_n = (unsigned)(g.N / GN), tiles_m = (unsigned)(g.M / GM);
  const unsigned t = gemm_tile(blockIdx.x, gridDim.x);
  // groups of 8 tile rows, column by column inside a group: the tiles an
  // XCD runs at once cover a square-ish block of C, so each A row panel and
  // each B column panel they read is shared by several of them
  const unsigned per_group = 8u * tiles_n, first = t / per_group * 8u;
  const unsigned gm = tiles_m - first < 8u ? tiles_m - first : 8u, w = t % per_group;
  const int m0 = (int)(first + w % gm) * GM, n0 = (int)(w / gm) * GN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 128;

  f32x16 acc[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

  // register stage of one K step: A as 4 float4 (rows tid/8 + 32 q, K
  // quad tid % 8); B as 8 float4 of B^T rows (TB = 1) or 32 values of one
  // column (TB = 0).  Buffer loads: one per-lane byte offset, the row and K
  // shifts in wave-uniform scalar offsets (the host keeps them below 2^31).
  const __amdgpu_buffer_rsrc_t RA = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(A), 0, 0x7fffffff, 0x00020000);
  const __amdgpu_buffer_rsrc_t RB = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(B), 0, 0x7fffffff, 0x00020000);
  const int vra = (int)((((tid >> 3) + 0LL) * g.lda + 4 * (tid & 7)) * 4);
  const int vrb = TB == 1 ? (int)((((tid >> 3) + 0LL) * g.ldb + 4 * (tid & 7)) * 4) : (n0 + 4 * lane) * 4;
  float4 ra[4];
  float rb[32];
  auto load = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int so = (int)(((long long)(m0 + 32 * q) * g.lda + k0) * 4);
      ra[q] = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(RA, vra, so, 0));
    }
    if constexpr (TB == 1) {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int so = (int)(((long long)(n0 + 32 * q) * g.ldb + k0) * 4);
        const float4 v = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(RB, vrb, so, 0));
        rb[4 * q] = v.x; rb[4 * q + 1] = v.y; rb[4 * q + 2] = v.z; rb[4 * q + 3] = v.w;
      }
    } else {
      // K x N: the wave takes K rows 8 w .. 8 w + 7, each lane 4 columns
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int so = (int)((long long)(k0 + 8 * wave + e) * g.ldb * 4);
        const float4 v = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(RB, vrb, so, 0));
        rb[4 * e] = v.x; rb[4 * e + 1] = v.y; rb[4 * e + 2] = v.z; rb[4 * e + 3] = v.w;
      }
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int row = (tid >> 3) + 32 * q, kq = 4 * (tid & 7);
      typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
      bf16x4 v = {(__bf16)ra[q].x, (__bf16)ra[q].y, (__bf16)ra[q].z, (__bf16)ra[q].w};
      *reinterpret_cast<bf16x4*>(&As[row][kq]) = v;
    }
    if constexpr (TB == 1) {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int row = (tid >> 3) + 32 * q, kq = 4 * (tid & 7);
        typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
        bf16x4 v = {(__bf16)rb[4 * q], (__bf16)rb[4 * q + 1], (__bf16)rb[4 * q + 2], (__bf16)rb[4 * q + 3]};
        *reinterpret_cast<bf16x4*>(&Bs[row][kq]) = v;
      }
    } else {
      // the 8 x 4 block transposed: column 4 lane + i gets its 8 K values
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        bf16x8 v;
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = (__bf16)rb[4 * e + i];
        *reinterpret_cast<bf16x8*>(&Bs[4 * lane + i][8 * wave]) = v;
      }
    }
  };

  load(0);
  store();
  __syncthreads();
  const int rl = lane & 31, kh = 8 * (lane >> 5);
  for (int k0 = 0; k0 < g.K; k0 += GK) {
    const bool more = k0 + GK < g.K;
    if (more) load(k0 + GK);
#pragma unroll
    for (int ks = 0; ks < GK; ks += 16) {
      bf16x8 a[2], b[4];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = *reinterpret_cast<const bf16x8*>(&As[wm + 32 * i + rl][ks + kh]);
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = *reinterpret_cast<const bf16x8*>(&Bs[wn + 32 * j + rl][ks + kh]);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
    if (more) {
      store();
      __syncthreads();
    }
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int m = m0 + wm + 32 * i + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int n = n0 + wn + 32 * j + (lane & 31);
        float* c = C + (long long)m * g.ldc + n;
        const float v = g.alpha * acc[i][j][r];
        *c = g.beta == 0.f ? v : v + g.beta * *c;
      }
}

__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float x) {
  // d/dx [x Phi(x)] = Phi(x) + x phi(x)
  return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * 0.39894228040143268f * expf(-0.5f * x * x);
}

__global__ __launch_bounds__(256) void k_bias_act(float* __restrict__ y, const float* __restrict__ bias,
                                                  long long rows, int cols, int act,
                                                  float* __restrict__ pre) {
  const long long n = rows * cols;
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (long long)gridDim.x * blockDim.x) {
    float v = y[k];
    if (bias) v += bias[k % cols];
    if (pre) pre[k] = v;
    y[k] = act == MCLBM_NN_GELU ? gelu(v) : v;
  }
}

__global__ __launch_bounds__(256) void k_act_backward(float* __restrict__ dy, const float* __restrict__ pre,
                                                      long long n, int act) {
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (long long)gridDim.x * blockDim.x)
    if (act == MCLBM_NN_GELU) dy[k] *= gelu_grad(pre[k]);
}

constexpr int kColChunk = 64;
constexpr int kRowGroups = 4;     // 256 threads = 64 columns x 4 row groups
constexpr int kRowsPerSlice = 256;

// partial[p][c] = sum of dy over rows [p*256, (p+1)*256) of column c
__global__ __launch_bounds__(256) void k_colsum_partial(const float* __restrict__ dy, long long rows, int cols,
                                                       float* __restrict__ partial) {
  __shared__ float red[kRowGroups][kColChunk];
  const int c = blockIdx.x * kColChunk + (threadIdx.x % kColChunk);
  const int gq = threadIdx.x / kColChunk;
  const long long r0 = (long long)blockIdx.y * kRowsPerSlice;
  float s = 0.f;
  if (c < cols)
    for (long long r = r0 + gq; r < std::min(rows, r0 + kRowsPerSlice); r += kRowGroups) s += dy[r * cols + c];
  red[gq][threadIdx.x % kColChunk] = s;
  __syncthreads();
  if (gq == 0 && c < cols) {
    float t = red[0][threadIdx.x];
    for (int q = 1; q < kRowGroups; ++q) t += red[q][threadIdx.x];
    partial[(long long)blockIdx.y * cols + c] = t;
  }
}

__global__ __launch_bounds__(256) void k_colsum_final(const float* __restrict__ partial, int slices, int cols,
                                                     float beta, float* __restrict__ db) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  float s = 0.f;
  for (int p = 0; p < slices; ++p) s += partial[(long long)p * cols + c];
  db[c] = beta == 0.f ? s : beta * db[c] + s;
}

constexpr int kMseBlock = 256;

__global__ __launch_bounds__(256) void k_mse_partial(const float* __restrict__ y, const float* __restrict__ t,
                                                    float* __restrict__ dy, long long n,
                                                    double* __restrict__ partial) {
  __shared__ double red[kMseBlock];
  const float inv = 2.0f / (float)n;
  double s = 0.0;
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (long long)gridDim.x * blockDim.x) {
    const float d = y[k] - t[k];
    dy[k] = inv * d;
    s += (double)d * (double)d;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = kMseBlock / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void k_mse_final(const double* __restrict__ partial, int nb, long long n, double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += partial[b];
  out[0] = s / (double)n;
}

__global__ __launch_bounds__(256) void k_adamw(float* __restrict__ w, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v, long long n,
                                              float lr, float b1, float b2, float eps, float wd,
                                              float c1, float c2) {
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (long long)gridDim.x * blockDim.x) {
    const float gk = g[k];
    const float mk = b1 * m[k] + (1.0f - b1) * gk;
    const float vk = b2 * v[k] + (1.0f - b2) * gk * gk;
    m[k] = mk;
    v[k] = vk;
    w[k] -= lr * ((mk / c1) / (sqrtf(vk / c2) + eps) + wd * w[k]);
  }
}

int nn_fail(int code, const char* msg) {
  mclbm_host::set_last_error(msg);
  return code;
}

int nn_check(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    mclbm_host::set_last_error(std::string(what) + ": " + hipGetErrorString(e));
    return MCLBM_EHIP;
  }
  return MCLBM_OK;
}

unsigned ew_blocks(long long n) { return (unsigned)std::max<long long>(1, std::min<long long>((n + 255) / 256, 65536)); }

}  // namespace

extern "C" {

int mclbm_nn_gemm(int32_t ta, int32_t tb, int32_t M, int32_t N, int32_t K, float alpha,
                  const float* A, int64_t lda, int64_t sa1, int64_t sa2,
                  const float* B, int64_t ldb, int64_t sb1, int64_t sb2,
                  float beta, float* C, int64_t ldc, int64_t sc1, int64_t sc2,
                  int32_t nb1, int32_t nb2, void* stream) {
  if (M < 1 || N < 1 || K < 1 || nb1 < 1 || nb2 < 1 || !A || !B || !C)
    return nn_fail(MCLBM_EINVAL, "gemm: bad sizes or NULL operand");
  if ((ta ? lda < M : lda < K) || (tb ? ldb < K : ldb < N) || ldc < N)
    return nn_fail(MCLBM_EINVAL, "gemm: leading dimension too small");
  if ((long long)nb1 * nb2 > 65535 || (M + BM - 1) / BM > 65535)
    return nn_fail(MCLBM_EINVAL, "gemm: more than 65535 batches or row tiles");
  GemmArgs g{ta, tb, M, N, K, nb2, alpha, beta, A, lda, sa1, sa2, B, ldb, sb1, sb2, C, ldc, sc1, sc2};
  const hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  // the large-tile kernel where the shape and alignment allow it
  auto a16 = [](const void* p) { return reinterpret_cast<uintptr_t>(p) % 16 == 0; };
  // (byte offsets within one batch entry below 2^31: the kernel addresses
  // its operands with 32-bit buffer offsets)
  const long long lim = (1LL << 31) - 64;
  const bool big = ta == 0 && M % GM == 0 && N % GN == 0 && K % GK == 0 && lda % 4 == 0 && sa1 % 4 == 0 &&
                   sa2 % 4 == 0 && a16(A) && (long long)(M / GM) * (N / GN) <= 0x7fffffff &&
                   (long long)M * lda * 4 < lim && (tb ? (long long)N * ldb * 4 : (long long)K * ldb * 4) < lim &&
                   ldb % 4 == 0 && sb1 % 4 == 0 && sb2 % 4 == 0 && a16(B);
  if (big) {
    dim3 grid((unsigned)((M / GM) * (N / GN)), 1, (unsigned)((long long)nb1 * nb2));
    if (tb)
      k_gemm_big<1><<<grid, 256, 0, st>>>(g);
    else
      k_gemm_big<0><<<grid, 256, 0, st>>>(g);
    return nn_check("k_gemm_big");
  }
  dim3 grid((N + BN - 1) / BN, (M + BM - 1) / BM, (unsigned)((long long)nb1 * nb2));
  k_gemm<<<grid, 256, 0, st>>>(g);
  return nn_check("k_gemm");
}

int mclbm_nn_bias_act(float* y, const float* bias, int64_t rows, int32_t cols, int32_t act, float* pre,
                      void* stream) {
  if (!y || rows < 0 || cols < 1 || (act != MCLBM_NN_ID && act != MCLBM_NN_GELU))
    return nn_fail(MCLBM_EINVAL, "bias_act: bad arguments");
  k_bias_act<<<ew_blocks(rows * cols), 256, 0, reinterpret_cast<hipStream_t>(stream)>>>(y, bias, rows, cols,
                                                                                         act, pre);
  return nn_check("k_bias_act");
}

int mclbm_nn_act_backward(float* dy, const float* pre, int64_t n, int32_t act, void* stream) {
  if (!dy || !pre || n < 0) return nn_fail(MCLBM_EINVAL, "act_backward: bad arguments");
  if (act == MCLBM_NN_ID) return MCLBM_OK;
  k_act_backward<<<ew_blocks(n), 256, 0, reinterpret_cast<hipStream_t>(stream)>>>(dy, pre, n, act);
  return nn_check("k_act_backward");
}

int64_t mclbm_nn_colsum_scratch(int64_t rows, int32_t cols) {
  return ((rows + kRowsPerSlice - 1) / kRowsPerSlice) * (int64_t)cols;
}

int mclbm_nn_colsum(const float* dy, float* db, int64_t rows, int32_t cols, float beta, float* scratch,
                    void* stream) {
  if (!dy || !db || !scratch || rows < 1 || cols < 1) return nn_fail(MCLBM_EINVAL, "colsum: bad arguments");
  const long long slices = (rows + kRowsPerSlice - 1) / kRowsPerSlice;
  if (slices > 65535) return nn_fail(MCLBM_EINVAL, "colsum: too many rows");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  k_colsum_partial<<<dim3((cols + kColChunk - 1) / kColChunk, (unsigned)slices), 256, 0, s>>>(dy, rows, cols,
                                                                                            scratch);
  int rc = nn_check("k_colsum_partial");
  if (rc) return rc;
  k_colsum_final<<<(cols + 255) / 256, 256, 0, s>>>(scratch, (int)slices, cols, beta, db);
  return nn_check("k_colsum_final");
}

int64_t mclbm_nn_mse_scratch(int64_t n) { return (int64_t)std::min<long long>((n + 255) / 256, 4096); }

int mclbm_nn_mse(const float* y, const float* t, float* dy, int64_t n, double* scratch, double* loss_out,
                 void* stream) {
  if (!y || !t || !dy || !scratch || !loss_out || n < 1) return nn_fail(MCLBM_EINVAL, "mse: bad arguments");
  const int nb = (int)mclbm_nn_mse_scratch(n);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  k_mse_partial<<<nb, kMseBlock, 0, s>>>(y, t, dy, n, scratch);
  int rc = nn_check("k_mse_partial");
  if (rc) return rc;
  k_mse_final<<<1, 64, 0, s>>>(scratch, nb, n, loss_out);
  return nn_check("k_mse_final");
}

int mclbm_nn_adamw(float* w, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                   float eps, float wd, int32_t t, void* stream) {
  if (!w || !g || !m || !v || n < 0 || t < 1) return nn_fail(MCLBM_EINVAL, "adamw: bad arguments");
  const float c1 = 1.0f - std::pow(b1, (float)t), c2 = 1.0f - std::pow(b2, (float)t);
  k_adamw<<<ew_blocks(n), 256, 0, reinterpret_cast<hipStream_t>(stream)>>>(w, g, m, v, n, lr, b1, b2, eps, wd,
                                                                            c1, c2);
  return nn_check("k_adamw");
}

}  // extern "C"
