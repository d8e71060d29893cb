// Device-side building blocks of the fused three-lattice MCLBM step for
// gfx950 (CDNA4, wave64): lattice constants, population storage, the A-A
// in-place access pattern with the cavity walls, and the per-node physics.
//
// Lattice (Section 2.d, Eqs 21 and 28): directions rest, E, N, W, S, NE, NW,
// SW, SE; lattice units dx = dt = 1, c_s^2 = 1/3.
//
// Memory layout in HBM (one copy updated in place by single steps; a second
// copy when two steps run per launch, each launch writing the copy it does
// not read):
//   pop[(l*9 + i)*plane + y*px + x]  l = 0 fluid f, 1 particles p, 2 theta g
//     (with two thermal lattices, Eq 19 for each phase: 2 fluid temperature
//     g, 3 particle temperature g2)
//   populations stored as deviations h = f - W_i rho_ref (rho_ref = 0 for g)
//   d2[k][y*px + x] = (phi - phi_ref, theta) of the step before, k = t & 1
//   d5[(lat*6 + wall*3 + slot)*px + x]  adiabatic-wall side buffer (see
//     below), one block of six rows per thermal lattice
//
// A-A pattern.  Even steps read the nine populations of a node from its own
// slots i and write the post-collision value of direction i into its own slot
// opp(i).  Odd steps read direction i from slot opp(i) of the upstream node
// x - e_i and write direction i into slot i of the downstream node x + e_i.
// Either way every thread reads exactly the slots it later writes, so one
// array suffices and no two threads touch the same slot.
//
// Walls (half-way, Eqs 34-36).  No-slip (Eq 34) is link bounce-back; the
// isothermal walls (Eq 35) use anti-bounce-back g_i = -g*_opp(i) + 2 W_i
// theta_w; in the A-A pattern both reduce to an access of the node's own
// slot.  The adiabatic walls (Eq 36) copy the unknown populations of the wall
// row from the row next to it in the same direction (after the isothermal
// rule at corners).  That copy reads slots that a neighbouring thread
// rewrites in the odd step, so even steps also store the three values the
// copy needs into the side buffer d5, which odd steps read; in odd steps the
// thread that produces a copied value also stores it into the wall row.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

namespace mclbm {

__host__ __device__ constexpr int ex(int i) {
  return (i == 1 || i == 5 || i == 8) ? 1 : ((i == 3 || i == 6 || i == 7) ? -1 : 0);
}
__host__ __device__ constexpr int ey(int i) {
  return (i == 2 || i == 5 || i == 6) ? 1 : ((i == 4 || i == 7 || i == 8) ? -1 : 0);
}
__host__ __device__ constexpr int opp(int i) {
  return i == 0 ? 0 : (i < 5 ? ((i + 1) % 4) + 1 : ((i - 3) % 4) + 5);
}
__host__ __device__ constexpr float wgt(int i) {
  return i == 0 ? 4.0f / 9.0f : (i < 5 ? 1.0f / 9.0f : 1.0f / 36.0f);
}
// exact weights in double precision (shift of the storage, exports)
__host__ __device__ constexpr double wgt_d(int i) {
  return i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
}
// side-buffer slot of a wall-row unknown: bottom row N, NE, NW; top S, SE, SW
__host__ __device__ constexpr int d5slot(int i) {
  return (i == 2 || i == 4) ? 0 : ((i == 5 || i == 8) ? 1 : 2);
}

static_assert(opp(1) == 3 && opp(2) == 4 && opp(5) == 7 && opp(6) == 8 &&
                  opp(7) == 5 && opp(8) == 6,
              "opposite directions");

// ---- population storage -------------------------------------------------
// Element access through a base pointer and an element index of type I
// (uint32_t when the population array is below 2 GiB, so that loads and
// stores take the scalar-base + 32-bit vector-offset form; uint64_t above).
template <class T, class I>
__device__ __forceinline__ const T* elem(const T* base, I idx) {
  if constexpr (sizeof(I) == 4)
    return reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) +
                                      (uint32_t)(idx * (uint32_t)sizeof(T)));
  else
    return base + idx;
}
template <class T, class I>
__device__ __forceinline__ T* elem(T* base, I idx) {
  return const_cast<T*>(elem(const_cast<const T*>(base), idx));
}

// FP32 deviations.  NTL / NTS mark the population loads / stores
// non-temporal (streamed past the caches), for cavities larger than the
// last-level cache.
// Buffer-resource forms (bld / bst) take a byte offset per lane (voff) and
// a wave-uniform byte offset (soff); policy bit 2 is the non-temporal hint.
template <bool NTL, bool NTS = NTL>
struct StorF32 {
  using T = float;
  static constexpr int kLdPol = NTL ? 2 : 0, kStPol = NTS ? 2 : 0;
  static __device__ __forceinline__ float ld(const T* p, float) {
    if constexpr (NTL) return __builtin_nontemporal_load(p);
    else return *p;
  }
  static __device__ __forceinline__ void st(T* p, float v, float) {
    if constexpr (NTS) __builtin_nontemporal_store(v, p);
    else *p = v;
  }
  static __device__ __forceinline__ float bld(__amdgpu_buffer_rsrc_t r, uint32_t voff,
                                              uint32_t soff, float) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, kLdPol));
  }
  static __device__ __forceinline__ void bst(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff,
                                             float v, float) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)voff, (int)soff, kStPol);
  }
};
// 16-bit deviations, FP16 scaled by a power of two per lattice (scale[l] on
// store, 1/scale[l] on load) so that typical deviations sit in the normal
// range, or BF16 (FP32's exponent range, scale 1).  Rounding to nearest even.
template <class H>
struct Half16;
template <>
struct Half16<__half> {
  static __device__ __forceinline__ float to_f(unsigned short b) {
    return __half2float(__ushort_as_half(b));
  }
  static __device__ __forceinline__ unsigned short from_f(float v) {
    return __half_as_ushort(__float2half_rn(v));
  }
};
template <>
struct Half16<__hip_bfloat16> {
  static __device__ __forceinline__ float to_f(unsigned short b) {
    return __uint_as_float((unsigned)b << 16);
  }
  static __device__ __forceinline__ unsigned short from_f(float v) {
    return __bfloat16_as_ushort(__float2bfloat16(v));
  }
};

template <class H, bool NTL, bool NTS = NTL>
struct Stor16 {
  using T = H;
  static constexpr int kLdPol = NTL ? 2 : 0, kStPol = NTS ? 2 : 0;
  static __device__ __forceinline__ float ld(const T* p, float inv) {
    unsigned short b;
    if constexpr (NTL) b = __builtin_nontemporal_load(reinterpret_cast<const unsigned short*>(p));
    else b = *reinterpret_cast<const unsigned short*>(p);
    return Half16<H>::to_f(b) * inv;
  }
  static __device__ __forceinline__ void st(T* p, float v, float sc) {
    const unsigned short b = Half16<H>::from_f(v * sc);
    if constexpr (NTS) __builtin_nontemporal_store(b, reinterpret_cast<unsigned short*>(p));
    else *reinterpret_cast<unsigned short*>(p) = b;
  }
  static __device__ __forceinline__ float bld(__amdgpu_buffer_rsrc_t r, uint32_t voff,
                                              uint32_t soff, float inv) {
    return Half16<H>::to_f(__builtin_amdgcn_raw_buffer_load_b16(r, (int)voff, (int)soff, kLdPol)) * inv;
  }
  static __device__ __forceinline__ void bst(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff,
                                             float v, float sc) {
    __builtin_amdgcn_raw_buffer_store_b16(Half16<H>::from_f(v * sc), r, (int)voff, (int)soff, kStPol);
  }
};
template <bool NTL, bool NTS = NTL>
using StorF16 = Stor16<__half, NTL, NTS>;
template <bool NTL, bool NTS = NTL>
using StorBF16 = Stor16<__hip_bfloat16, NTL, NTS>;

// Reciprocal: hardware estimate refined by one Newton step (~0.5 ulp),
// instead of the long IEEE division sequence.
__device__ __forceinline__ float frcp(float x) {
  const float r = __builtin_amdgcn_rcpf(x);
  return fmaf(r, fmaf(-x, r, 1.0f), r);
}
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
// x^y for x >= 0 as 2^(y log2 x), with the hardware base-2 logarithm and
// exponential (a few ulp; the correctly rounded library power costs ~150
// instructions, a third of the node update).  x = 0 gives 0.
__device__ __forceinline__ float fpow(float x, float y) {
  return __builtin_amdgcn_exp2f(y * __builtin_amdgcn_logf(x));
}

// ---- kernel parameters (kernarg, by value) -------------------------------
struct StepParams {
  int nx, ny, px, nl;    // nl: lattices, 3 or 4 (two thermal lattices)
  long long plane;       // elements per population plane
  float scale[3];        // storage scale per lattice (1 for FP32)
  float inv_scale[3];
  // reference state and relaxation
  float rho_f_ref, rho_p_ref, dref_p;  // dref_p = rho_p_ref - R phi0
  float rho_p0;                        // R phi0
  float tau_f, omega_f;
  // properties (Eqs 7-11, 22-24)
  float invR, Rm1, crc, crb, Ck, alpha3;
  float tp_a, tp_b;      // tau_p = tau_f + tp_a rho_m (tp_b + 222.4 phi)/r_rho
  float G_L;             // g beta dT in lattice units
  float omega_thf, tau_thf;  // relaxation of the fluid thermal lattice (nl = 4)
  // slip forces (Table 1) in lattice units, switches and scales folded in
  float cB;              // Brownian
  float cT, kfp, A1, A2; // thermophoresis
  float dT_T0;
  float cS;              // Saffman
  float cM, cR;          // Magnus, particle rotation
  float cG;              // settling per particle mass, (1 - 1/R) g
  float cRe, cD;         // drag: Re_d and Stokes rate coefficients
  unsigned force_on;     // bit k set when force k has a non-zero coefficient
  unsigned flags;        // bit 0: f and p relax to one common velocity
};

// ---- A-A access ------------------------------------------------------------
// Arrays below 2 GiB are accessed through a buffer resource: one per-lane
// byte offset shared by all 27 accesses of a node, and a wave-uniform scalar
// offset per plane that also carries the neighbour shift (x and row), so no
// per-access address arithmetic runs on the vector units.  Lanes next to a
// wall take a separate, exec-masked path, which waves away from the walls
// skip.  Larger arrays use 64-bit pointer arithmetic.
// Buffer resource over the population array (raw, byte-addressed, range
// checked against its size).
template <class T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t pop_rsrc(const T* pop, const StepParams& P) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(pop), 0,
                                           (int)(9u * (uint32_t)P.nl * (uint32_t)P.plane * (uint32_t)sizeof(T)),
                                           0x00020000);
}
// wave-uniform byte offset of plane q shifted by (dx, dy) nodes
template <class T>
__device__ __forceinline__ uint32_t soff(const StepParams& P, int q, int dx, int dy) {
  return (uint32_t)(q * (int)P.plane + dy * P.px + dx) * (uint32_t)sizeof(T);
}

// ---- read the nine populations of each lattice ------------------------------
template <bool ODD, class S, class I, int NL = 3>
__device__ __forceinline__ void load_node(const StepParams& P,
                                          const typename S::T* __restrict__ pop,
                                          const float* __restrict__ d5, int x,
                                          int y, float f[9], float p[9],
                                          float g[9], float g2[9] = nullptr) {
  using T = typename S::T;
  const I px = (I)P.px, pl = (I)P.plane;
  const I n = (I)y * px + (I)x;
  const bool xl = x == 0, xr = x == P.nx - 1, yb = y == 0, yt = y == P.ny - 1;
  if constexpr (sizeof(I) == 4) {
    const __amdgpu_buffer_rsrc_t R = pop_rsrc(pop, P);
    const uint32_t vo = (uint32_t)n * (uint32_t)sizeof(T);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      if (!ODD) {
        f[i] = S::bld(R, vo, soff<T>(P, i, 0, 0), P.inv_scale[0]);
        p[i] = S::bld(R, vo, soff<T>(P, 9 + i, 0, 0), P.inv_scale[1]);
        g[i] = S::bld(R, vo, soff<T>(P, 18 + i, 0, 0), P.inv_scale[2]);
        if constexpr (NL == 4) g2[i] = S::bld(R, vo, soff<T>(P, 27 + i, 0, 0), P.inv_scale[2]);
      } else {
        const bool outx = (ex(i) == 1 && xl) || (ex(i) == -1 && xr);
        const bool outy = (ey(i) == 1 && yb) || (ey(i) == -1 && yt);
        if (!(outx || outy)) {
          // upstream node x - e_i, slot opp(i)
          f[i] = S::bld(R, vo, soff<T>(P, opp(i), -ex(i), -ey(i)), P.inv_scale[0]);
          p[i] = S::bld(R, vo, soff<T>(P, 9 + opp(i), -ex(i), -ey(i)), P.inv_scale[1]);
          g[i] = S::bld(R, vo, soff<T>(P, 18 + opp(i), -ex(i), -ey(i)), P.inv_scale[2]);
          if constexpr (NL == 4) g2[i] = S::bld(R, vo, soff<T>(P, 27 + opp(i), -ex(i), -ey(i)), P.inv_scale[2]);
        } else {
          // wall link: own slot i (bounce-back); the thermal lattices by
          // the wall rules (side buffer block 6 l for thermal lattice l)
          f[i] = S::bld(R, vo, soff<T>(P, i, 0, 0), P.inv_scale[0]);
          p[i] = S::bld(R, vo, soff<T>(P, 9 + i, 0, 0), P.inv_scale[1]);
#pragma unroll
          for (int l = 0; l < NL - 2; ++l) {
            float* h = l == 0 ? g : g2;
            if (outy) {
              h[i] = d5[(6 * l + (ey(i) == 1 ? 0 : 3) + d5slot(i)) * P.px + x];
            } else {
              const float v = S::bld(R, vo, soff<T>(P, 18 + 9 * l + i, 0, 0), P.inv_scale[2]);
              h[i] = (xl ? wgt(i) : -wgt(i)) - v;
            }
          }
        }
      }
    }
    return;
  } else {
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      if (!ODD) {
        f[i] = S::ld(elem(pop, pl * (I)i + n), P.inv_scale[0]);
        p[i] = S::ld(elem(pop, pl * (I)(9 + i) + n), P.inv_scale[1]);
        g[i] = S::ld(elem(pop, pl * (I)(18 + i) + n), P.inv_scale[2]);
        if constexpr (NL == 4) g2[i] = S::ld(elem(pop, pl * (I)(27 + i) + n), P.inv_scale[2]);
      } else {
        const bool outx = (ex(i) == 1 && xl) || (ex(i) == -1 && xr);
        const bool outy = (ey(i) == 1 && yb) || (ey(i) == -1 && yt);
        const bool out = outx || outy;
        // inside: upstream node's slot opp(i); wall link: own slot i
        const I up = n - (I)ex(i) - (I)ey(i) * px;  // wraps only when unused
        const I a = out ? (pl * (I)i + n) : (pl * (I)opp(i) + up);
        f[i] = S::ld(elem(pop, a), P.inv_scale[0]);
        p[i] = S::ld(elem(pop, pl * (I)9 + a), P.inv_scale[1]);
#pragma unroll
        for (int l = 0; l < NL - 2; ++l) {
          float* h = l == 0 ? g : g2;
          const I tb = pl * (I)(18 + 9 * l);
          if (i == 0) {
            h[i] = S::ld(elem(pop, tb + a), P.inv_scale[2]);
          } else if (outy) {
            h[i] = d5[(6 * l + (ey(i) == 1 ? 0 : 3) + d5slot(i)) * P.px + x];
          } else {
            const float v = S::ld(elem(pop, tb + a), P.inv_scale[2]);
            h[i] = outx ? (xl ? wgt(i) : -wgt(i)) - v : v;
          }
        }
      }
    }
  }
}

// ---- write the post-collision populations -----------------------------------
// side buffer for the adiabatic copy of the next (odd) step, block db
__device__ __forceinline__ void store_side(const StepParams& P, float* __restrict__ d5, int db, int x, int y,
                                           const float g[9]) {
  const int px = P.px, nx = P.nx, ny = P.ny;
  const bool xl = x == 0, xr = x == nx - 1, yb = y == 0, yt = y == ny - 1;
  float* d = d5 + (size_t)db * px;
  if (yb) {
    d[0 * px + x] = g[2];
    if (!xr) d[1 * px + x + 1] = g[5];
    if (!xl) d[2 * px + x - 1] = g[6];
  }
  if (y == 1) {
    if (xl) d[1 * px + 0] = wgt(5) - g[7];
    if (xr) d[2 * px + nx - 1] = -wgt(6) - g[8];
  }
  if (yt) {
    d[3 * px + x] = g[4];
    if (!xr) d[4 * px + x + 1] = g[8];
    if (!xl) d[5 * px + x - 1] = g[7];
  }
  if (y == ny - 2) {
    if (xl) d[4 * px + 0] = wgt(8) - g[6];
    if (xr) d[5 * px + nx - 1] = -wgt(7) - g[5];
  }
}

template <bool ODD, class S, class I, int NL = 3>
__device__ __forceinline__ void store_node(const StepParams& P,
                                           typename S::T* __restrict__ pop,
                                           float* __restrict__ d5, int x, int y,
                                           const float f[9], const float p[9],
                                           const float g[9], const float g2[9] = nullptr) {
  using T = typename S::T;
  const I px = (I)P.px, pl = (I)P.plane;
  const I n = (I)y * px + (I)x;
  const int nx = P.nx, ny = P.ny;
  const bool xl = x == 0, xr = x == nx - 1, yb = y == 0, yt = y == ny - 1;
  if constexpr (sizeof(I) == 4) {
    const __amdgpu_buffer_rsrc_t R = pop_rsrc(pop, P);
    const uint32_t vo = (uint32_t)n * (uint32_t)sizeof(T);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      if (!ODD) {
        S::bst(R, vo, soff<T>(P, opp(i), 0, 0), f[i], P.scale[0]);
        S::bst(R, vo, soff<T>(P, 9 + opp(i), 0, 0), p[i], P.scale[1]);
        S::bst(R, vo, soff<T>(P, 18 + opp(i), 0, 0), g[i], P.scale[2]);
        if constexpr (NL == 4) S::bst(R, vo, soff<T>(P, 27 + opp(i), 0, 0), g2[i], P.scale[2]);
      } else {
        const bool outx = (ex(i) == 1 && xr) || (ex(i) == -1 && xl);
        const bool outy = (ey(i) == 1 && yt) || (ey(i) == -1 && yb);
        if (!(outx || outy)) {
          // downstream node x + e_i, slot i
          S::bst(R, vo, soff<T>(P, i, ex(i), ey(i)), f[i], P.scale[0]);
          S::bst(R, vo, soff<T>(P, 9 + i, ex(i), ey(i)), p[i], P.scale[1]);
#pragma unroll
          for (int l = 0; l < NL - 2; ++l) {
            const float gv = l == 0 ? g[i] : g2[i];
            S::bst(R, vo, soff<T>(P, 18 + 9 * l + i, ex(i), ey(i)), gv, P.scale[2]);
            // the wall row takes the same value (copy of the adiabatic wall)
            if ((ey(i) == 1 && yb) || (ey(i) == -1 && yt))
              S::bst(R, vo, soff<T>(P, 18 + 9 * l + i, ex(i), 0), gv, P.scale[2]);
          }
        } else {
          // wall link: own slot opp(i)
          S::bst(R, vo, soff<T>(P, opp(i), 0, 0), f[i], P.scale[0]);
          S::bst(R, vo, soff<T>(P, 9 + opp(i), 0, 0), p[i], P.scale[1]);
          if (!outy) {
#pragma unroll
            for (int l = 0; l < NL - 2; ++l) {
              // isothermal wall: anti-bounce-back into the own slot opp(i)
              const float v = (ex(i) == -1 ? wgt(i) : -wgt(i)) - (l == 0 ? g[i] : g2[i]);
              const int q = 18 + 9 * l + opp(i);
              S::bst(R, vo, soff<T>(P, q, 0, 0), v, P.scale[2]);
              // corner: the wall row next to this one copies it
              if (ey(opp(i)) == 1 && y == 1) S::bst(R, vo, soff<T>(P, q, 0, -1), v, P.scale[2]);
              if (ey(opp(i)) == -1 && y == ny - 2) S::bst(R, vo, soff<T>(P, q, 0, 1), v, P.scale[2]);
            }
          }
          // out through an adiabatic wall: the value leaves the domain
        }
      }
    }
  } else {
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      if (!ODD) {
        S::st(elem(pop, pl * (I)opp(i) + n), f[i], P.scale[0]);
        S::st(elem(pop, pl * (I)(9 + opp(i)) + n), p[i], P.scale[1]);
        S::st(elem(pop, pl * (I)(18 + opp(i)) + n), g[i], P.scale[2]);
        if constexpr (NL == 4) S::st(elem(pop, pl * (I)(27 + opp(i)) + n), g2[i], P.scale[2]);
      } else {
        const bool outx = (ex(i) == 1 && xr) || (ex(i) == -1 && xl);
        const bool outy = (ey(i) == 1 && yt) || (ey(i) == -1 && yb);
        const bool out = outx || outy;
        const I down = n + (I)ex(i) + (I)ey(i) * px;  // wraps only when unused
        const I a = out ? (pl * (I)opp(i) + n) : (pl * (I)i + down);
        S::st(elem(pop, a), f[i], P.scale[0]);
        S::st(elem(pop, pl * (I)9 + a), p[i], P.scale[1]);
#pragma unroll
        for (int l = 0; l < NL - 2; ++l) {
          const float gv = l == 0 ? g[i] : g2[i];
          const I tb = pl * (I)(18 + 9 * l);
          if (i == 0) {
            S::st(elem(pop, tb + a), gv, P.scale[2]);
          } else if (!out) {
            S::st(elem(pop, tb + a), gv, P.scale[2]);
            if ((ey(i) == 1 && yb) || (ey(i) == -1 && yt))
              S::st(elem(pop, tb + pl * (I)i + n + (I)ex(i)), gv, P.scale[2]);
          } else if (!outy) {
            const float v = (ex(i) == -1 ? wgt(i) : -wgt(i)) - gv;
            S::st(elem(pop, tb + a), v, P.scale[2]);
            if (ey(opp(i)) == 1 && y == 1) S::st(elem(pop, tb + a - px), v, P.scale[2]);
            if (ey(opp(i)) == -1 && y == ny - 2) S::st(elem(pop, tb + a + px), v, P.scale[2]);
          }
        }
      }
    }
  }
  if (!ODD) {
    store_side(P, d5, 0, x, y, g);
    if constexpr (NL == 4) store_side(P, d5, 6, x, y, g2);
  }
}

// ---- BGK collision with forcing in deviation form (Eqs 18-19, 26-27) ------
// h* = h + omega (h_eq - h) + S,
// h_eq_i = W_i [d + a (3 e.u + 4.5 (e.u)^2 - 1.5 u^2)], S_i = 3 W_i e_i.F,
// with d = sum h the density deviation, a the full density and j = a u the
// first moment (for g: d = a = theta, j = theta u_ns).
// The weights 1/9 and 1/36 are inexact in binary floating point, so the
// textbook per-direction form leaks mass and momentum by ~1e-8 of the state
// per step.  Here the equilibrium is assembled from its symmetric and
// antisymmetric parts per direction pair so that sum h_eq = d and
// sum h_eq e = j (and sum S = 0, sum S e = F) hold by construction: the
// diagonal pairs take their exact-weight values, the axis pairs take what
// remains of j/2, and the rest population what remains of d.
__device__ __forceinline__ void collide(float h[9], float d, float a, float jx,
                                        float jy, float ux, float uy,
                                        float omega, float Fx, float Fy) {
  constexpr float W1 = 1.0f / 9.0f, W5 = 1.0f / 36.0f;
  const float base = fmaf(-1.5f * a, fmaf(ux, ux, uy * uy), d);
  const float a45 = 4.5f * a;
  const float up = ux + uy, um = ux - uy;
  // symmetric parts of the pairs (1,3), (2,4), (5,7), (8,6)
  const float S1 = W1 * fmaf(a45 * ux, ux, base);
  const float S2 = W1 * fmaf(a45 * uy, uy, base);
  const float S5 = W5 * fmaf(a45 * up, up, base);
  const float S8 = W5 * fmaf(a45 * um, um, base);
  // antisymmetric parts: diagonals exact-weight, axes close the momentum
  const float A5 = (3.0f * W5) * (jx + jy);
  const float A8 = (3.0f * W5) * (jx - jy);
  const float A1 = fmaf(0.5f, jx, -(A5 + A8));
  const float A2 = fmaf(0.5f, jy, A8 - A5);
  const float S0 = d - 2.0f * ((S1 + S2) + (S5 + S8));
  // forcing, same construction
  const float B5 = (3.0f * W5) * (Fx + Fy);
  const float B8 = (3.0f * W5) * (Fx - Fy);
  const float B1 = fmaf(0.5f, Fx, -(B5 + B8));
  const float B2 = fmaf(0.5f, Fy, B8 - B5);
  h[0] = fmaf(omega, S0 - h[0], h[0]);
  h[1] = fmaf(omega, (S1 + A1) - h[1], h[1]) + B1;
  h[3] = fmaf(omega, (S1 - A1) - h[3], h[3]) - B1;
  h[2] = fmaf(omega, (S2 + A2) - h[2], h[2]) + B2;
  h[4] = fmaf(omega, (S2 - A2) - h[4], h[4]) - B2;
  h[5] = fmaf(omega, (S5 + A5) - h[5], h[5]) + B5;
  h[7] = fmaf(omega, (S5 - A5) - h[7], h[7]) - B5;
  h[8] = fmaf(omega, (S8 + A8) - h[8], h[8]) + B8;
  h[6] = fmaf(omega, (S8 - A8) - h[6], h[6]) - B8;
}

struct NodeMoments {
  float drf, jxf, jyf, drp, jxp, jyp, th;
};

__device__ __forceinline__ NodeMoments moments(const float f[9], const float p[9],
                                               const float g[9]) {
  NodeMoments m;
  m.drf = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + (f[7] + f[8])));
  m.jxf = (f[1] - f[3]) + ((f[5] - f[6]) + (f[8] - f[7]));
  m.jyf = (f[2] - f[4]) + ((f[5] - f[8]) + (f[6] - f[7]));
  m.drp = ((p[0] + p[1]) + (p[2] + p[3])) + ((p[4] + p[5]) + (p[6] + (p[7] + p[8])));
  m.jxp = (p[1] - p[3]) + ((p[5] - p[6]) + (p[8] - p[7]));
  m.jyp = (p[2] - p[4]) + ((p[5] - p[8]) + (p[6] - p[7]));
  m.th = ((g[0] + g[1]) + (g[2] + g[3])) + ((g[4] + g[5]) + (g[6] + (g[7] + g[8])));
  return m;
}

// ---- one node: moments, properties, slip forces, collision ---------------
// gphi, gth: central-difference gradients of the previous step's fields.
// Returns the fields this step stores for the next step's gradients.
// NL = 4: two thermal lattices (Eq 19 for each phase), g for the fluid and
// g2 for the particles; the suspension temperature is their heat-capacity
// weighted mean (Eq 33) and drives buoyancy and thermophoresis.
template <int NL = 3>
__device__ __forceinline__ float2 node_update(const StepParams& P, float f[9],
                                              float p[9], float g[9],
                                              float gphix, float gphiy,
                                              float gthx, float gthy, float g2[9] = nullptr) {
  const NodeMoments m = moments(f, p, g);
  // S1/S2: Eqs 29-32 (partial densities; mass-averaged mixture velocity)
  const float rho_f = P.rho_f_ref + m.drf;
  const float rho_p = P.rho_p_ref + m.drp;
  const float irf = frcp(rho_f);
  const float uxf = m.jxf * irf, uyf = m.jyf * irf;
  const bool empty = !(rho_p > 1e-12f);
  const float irp = empty ? 0.0f : frcp(rho_p);
  const float uxp = empty ? uxf : m.jxp * irp;
  const float uyp = empty ? uyf : m.jyp * irp;
  const float rho_m = rho_f + rho_p;
  const float irm = frcp(rho_m);
  const float uxn = (m.jxf + m.jxp) * irm, uyn = (m.jyf + m.jyp) * irm;

  // S3: Eqs 7-11 as ratios to the base fluid; Eq 23 for tau_p; Eq 24
  const float phi = rho_p * P.invR;
  const float phic = fmaxf(phi, 0.0f);
  const float r_rho = fmaf(phi, P.Rm1, 1.0f);
  const float r_rhoc = fmaf(phi, P.crc, 1.0f);
  const float r_beta = fmaf(phi, P.crb, 1.0f);
  const float r_mu = fmaf(phi, fmaf(222.4f, phi, 4.93f), 1.0f);
  const float r_k = fmaf(P.Ck, fpow(phic, 0.764f), 1.0f);
  const float ir_rho = frcp(r_rho);
  float tau_p = P.tau_f + P.tp_a * rho_m * fmaf(222.4f, phi, P.tp_b) * ir_rho;
  tau_p = fminf(fmaxf(tau_p, 0.505f), 5.0f);
  if (empty) tau_p = P.tau_f;
  const float tau_th = fmaf(P.alpha3 * r_k, frcp(r_rhoc), 0.5f);
  // temperature of the suspension: the single thermal lattice, or Eq 33
  // over the two (volume fractions 1 - phi and phi, heat capacities per
  // volume in the ratio 1 : 1 + crc)
  float th = m.th, thp = 0.0f;
  if constexpr (NL == 4) {
    thp = ((g2[0] + g2[1]) + (g2[2] + g2[3])) + ((g2[4] + g2[5]) + (g2[6] + (g2[7] + g2[8])));
    th = fmaf(phic, fmaf(P.crc + 1.0f, thp, -m.th), m.th) * frcp(fmaf(phic, P.crc, 1.0f));
  }

  // S5: forces.  The fluid carries buoyancy (Eq 20) and the net weight of
  // the particles relative to the uniform suspension; every interaction
  // force acts on both lattices with opposite signs.
  const float dp_true = m.drp + P.dref_p;          // rho_p - R phi0
  const float Fbuoy = rho_m * r_beta * P.G_L * th;  // Eq 20, beta_ns of Eq 9
  float Fpx = 0.0f, Fpy = 0.0f;
  if (!empty) {
    const unsigned on = P.force_on;
    const float wx = uxf - uxp, wy = uyf - uyp;
    const float wn = fsqrt(fmaf(wx, wx, wy * wy));
    const float upn = fsqrt(fmaf(uxp, uxp, uyp * uyp));
    const float r_mu2 = r_mu * r_mu;
    const float ir_mu = frcp(r_mu);
    float aix = 0.0f, aiy = 0.0f;  // interaction forces per particle mass
    if (on & 2u) {  // Brownian, down the phi gradient
      const float Tr = fmaf(P.dT_T0, th, 1.0f);
      const float c = -P.cB * Tr * Tr * (ir_mu * ir_mu);
      aix = fmaf(c, gphix, aix);
      aiy = fmaf(c, gphiy, aiy);
    }
    if (on & 4u) {  // thermophoresis, down the temperature gradient
      const float Tr = fmaf(P.dT_T0, th, 1.0f);
      const float ks = P.kfp * r_k;
      const float CT = P.A2 * (ks + P.A1) * frcp(fmaf(2.0f, ks + P.A1, 1.0f));
      const float c = -P.cT * CT * r_mu2 * ir_rho * frcp(Tr);
      aix = fmaf(c, gthx, aix);
      aiy = fmaf(c, gthy, aiy);
    }
    if (on & 8u) {  // Saffman lift, along the rotated slip
      const float c = P.cS * fsqrt(r_mu * r_rho * upn);
      aix = fmaf(-c, wy, aix);
      aiy = fmaf(c, wx, aiy);
    }
    if (on & 16u) {  // Magnus (opposes the slip) + particle rotation
      const float vmx = 0.5f * (uxf + uxp), vmy = 0.5f * (uyf + uyp);
      const float cm = -0.5f * P.cM * fsqrt(fmaf(vmx, vmx, vmy * vmy));
      const float iwn = wn > 0.0f ? frcp(wn) : 0.0f;
      const float cr = P.cR * r_mu * ir_rho * upn * iwn;
      aix = fmaf(cm, wx, fmaf(-cr, wy, aix));
      aiy = fmaf(cm, wy, fmaf(cr, wx, aiy));
    }
    const float aGy = -P.cG;  // settling per particle mass (0 when off)
    if (on & 1u) {
      // Drag integrated exactly over the step (stiff: kappa ~ 1e4).  Its
      // mean combined with the other particle forces is
      //   F^p = rho_p [phi1 (a_int + beta w) + beta phi2 Fext_f / rho_f
      //               + a_G (r + phi1) / (1 + r)],
      // r = rho_p/rho_f, kappa = beta (1 + r), phi1 = (1 - e^-kappa)/kappa,
      // phi2 = (1 - phi1)/kappa, a_int the interaction forces per particle
      // mass, a_G settling, Fext_f buoyancy plus the fluid's gravity
      // reference.  Written this way no large terms cancel (the reacting
      // forces and the drag nearly balance each other).
      const float r = rho_p * irf;
      const float Red = P.cRe * wn * ir_mu;
      const float beta = P.cD * r_mu * fmaf(0.15f, fpow(Red, 0.687f), 1.0f);
      const float kap = beta * (1.0f + r);
      float ph1, ph2;
      if (kap < 0.05f) {  // Taylor series, truncation < 1e-8
        ph1 = fmaf(kap, fmaf(kap, fmaf(kap, -1.0f / 24.0f, 1.0f / 6.0f), -0.5f), 1.0f);
        ph2 = fmaf(kap, fmaf(kap, fmaf(kap, -1.0f / 120.0f, 1.0f / 24.0f), -1.0f / 6.0f), 0.5f);
      } else {
        const float ik = frcp(kap);
        ph1 = -expm1f(-kap) * ik;
        ph2 = (1.0f - ph1) * ik;
      }
      // The gravity terms (settling, fluid reference) combine, with
      // beta phi2 = (1 - phi1)/(1 + r), into
      //   -cG [ (rho_p - R phi0) + phi1 (R phi0 + rho_f) ] / rho_m
      // and buoyancy into (1 - phi1) Fbuoy / rho_m: no cancellation.
      const float om1 = kap < 0.05f ? kap * ph2 : 1.0f - ph1;
      const float ext = fmaf(om1, Fbuoy, -P.cG * fmaf(ph1, P.rho_p0 + rho_f, dp_true)) * irm;
      Fpx = rho_p * ph1 * fmaf(beta, wx, aix);
      Fpy = rho_p * fmaf(ph1, fmaf(beta, wy, aiy), ext);
    } else {
      Fpx = rho_p * aix;
      Fpy = rho_p * (aiy + aGy);
    }
  }
  const float Ffx = -Fpx;
  const float Ffy = fmaf(-P.cG, dp_true, Fbuoy) - Fpy;

  // S6: collisions; f and p relax to their own velocities, g to u_ns
  float ufx = uxf, ufy = uyf, upx = uxp, upy = uyp;
  float jfx = m.jxf, jfy = m.jyf;
  float jpx = empty ? rho_p * uxf : m.jxp, jpy = empty ? rho_p * uyf : m.jyp;
  const float omega_p = frcp(tau_p);
  if (P.flags & 1u) {
    // alternative reading: one common equilibrium velocity weighted by
    // rho / tau, which conserves the mixture momentum of the collision
    const float wf = rho_f * P.omega_f, wp = empty ? 0.0f : rho_p * omega_p;
    const float iw = frcp(wf + wp);
    ufx = upx = fmaf(wf, uxf, wp * uxp) * iw;
    ufy = upy = fmaf(wf, uyf, wp * uyp) * iw;
    jfx = rho_f * ufx; jfy = rho_f * ufy;
    jpx = rho_p * ufx; jpy = rho_p * ufy;
  }
  collide(f, m.drf, rho_f, jfx, jfy, ufx, ufy, P.omega_f, Ffx, Ffy);
  collide(p, m.drp, rho_p, jpx, jpy, upx, upy, omega_p, Fpx, Fpy);
  if constexpr (NL == 4) {
    // each phase's thermal lattice relaxes to its own velocity; the fluid's
    // with the base-fluid diffusivity, the particles' with the relaxation
    // time that makes the mass-weighted sum of Eq 24 equal tau_theta of the
    // suspension
    const float thf = m.th;
    collide(g, thf, thf, thf * uxf, thf * uyf, uxf, uyf, P.omega_thf, 0.0f, 0.0f);
    float tau_tp = P.tau_thf;
    if (!empty) tau_tp = fminf(fmaxf(fmaf(tau_th - P.tau_thf, rho_m * irp, P.tau_thf), 0.505f), 5.0f);
    collide(g2, thp, thp, thp * uxp, thp * uyp, uxp, uyp, frcp(tau_tp), 0.0f, 0.0f);
  } else {
    collide(g, th, th, th * uxn, th * uyn, uxn, uyn, frcp(tau_th), 0.0f, 0.0f);
  }
  return make_float2(m.drp * P.invR, th);
}

}  // namespace mclbm
