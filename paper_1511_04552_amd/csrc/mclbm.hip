// libmclbm: the fused three-lattice MCLBM time step for MI355X (gfx950) and
// its C ABI (include/mclbm.h).
//
// Kernels
//   k_init      initial equilibrium state (Eqs 26-27) and the lag field
//   k_step      the fused hot path, one launch per time step: A-A load with
//               streaming and walls (Eqs 34-36), moments (Eqs 29-32),
//               properties (Eqs 7-11, 22-24), lagged gradients, slip forces
//               (Table 1, Eqs 6, 20), BGK collision of three lattices
//               (Eqs 18-19), A-A store
//   k_step2     the same physics for an even and the following odd step in
//               one launch, between two population copies (large cavities)
//   k_step_batch  one launch per step over a batch of uneven cavities
//   k_step2_batch two steps per launch over such a batch (tiles of k_step2)
//   k_step_cavity many steps per launch over a batch of small cavities, one
//               workgroup per cavity
//   k_nusselt   FP64 wall-Nusselt reduction
//   k_residual  FP64 relative change of u_ns and theta (steady-state test)
//   k_*_batch   the same reductions for every active cavity of a batch
//   k_export    FP64 moments / populations of the current state
//   k_copy      plain streaming copy, bandwidth and counter calibration
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "mclbm.h"
#include "lbm_device.h"

using namespace mclbm;

// ===========================================================================
// Kernels
// ===========================================================================

template <class S, int NL>
__global__ __launch_bounds__(256) void k_init(StepParams P,
                                              typename S::T* __restrict__ pop,
                                              const double* __restrict__ dev_p,
                                              double dev_f,
                                              float2* __restrict__ d2prev) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  if (x >= P.nx || y >= P.ny) return;
  const long long n = (long long)y * P.px + x;
  const double dp = dev_p[(long long)y * P.nx + x];
  float f[9], p[9], g[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const double w = wgt_d(i);
    f[i] = (float)(w * dev_f);
    p[i] = (float)(w * dp);
    g[i] = 0.0f;
    S::st(pop + P.plane * i + n, f[i], P.scale[0]);
    S::st(pop + P.plane * (9 + i) + n, p[i], P.scale[1]);
    S::st(pop + P.plane * (18 + i) + n, g[i], P.scale[2]);
    if constexpr (NL == 4) S::st(pop + P.plane * (27 + i) + n, 0.0f, P.scale[2]);
  }
  // the lag field holds what the first step would have stored (theta = 0
  // on every thermal lattice, so the suspension temperature is 0 too)
  float fl[9], pl[9], gl[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    fl[i] = S::ld(pop + P.plane * i + n, P.inv_scale[0]);
    pl[i] = S::ld(pop + P.plane * (9 + i) + n, P.inv_scale[1]);
    gl[i] = S::ld(pop + P.plane * (18 + i) + n, P.inv_scale[2]);
  }
  const NodeMoments m = moments(fl, pl, gl);
  d2prev[n] = make_float2(m.drp * P.invR, m.th);
}

// Workgroups are dealt round-robin to the 8 XCDs of the chip, each with its
// own L2.  The step kernel runs on a 1-D grid and maps workgroup b to tile
// start(b % 8) + b / 8, so that each XCD sweeps one contiguous band of rows:
// the neighbour rows an odd step and the lag-field stencil touch are then
// mostly in the same L2.
__device__ __forceinline__ unsigned xcd_tile(unsigned b, unsigned nb) {
  const unsigned q = nb >> 3, r = nb & 7u, k = b & 7u;
  return k * q + (k < r ? k : r) + (b >> 3);
}

// S4: central differences of the previous step's (phi, theta); zero-flux
// mirror ghosts for phi on all walls and for theta on the adiabatic walls,
// linear ghosts 2 theta_w - theta through the isothermal walls.  Returns
// (dphi/dx, dphi/dy, dtheta/dx, dtheta/dy).
__device__ __forceinline__ void wall_ghosts(float2 c, float2 vE, float2 vW, float2 vN, float2 vS,
                                            bool xl, bool xr, bool yb, bool yt, float4& gr) {
  vE = xr ? c : vE;
  vW = xl ? c : vW;
  vN = yt ? c : vN;
  vS = yb ? c : vS;
  const float thE = xr ? (-1.0f - c.y) : vE.y;
  const float thW = xl ? (1.0f - c.y) : vW.y;
  gr = make_float4(0.5f * (vE.x - vW.x), 0.5f * (vN.x - vS.x), 0.5f * (thE - thW), 0.5f * (vN.y - vS.y));
}

__device__ __forceinline__ void lag_gradients(const StepParams& P, const float2* __restrict__ d2p, int x,
                                              int y, float4& gr) {
  const long long n = (long long)y * P.px + x;
  const bool xl = x == 0, xr = x == P.nx - 1, yb = y == 0, yt = y == P.ny - 1;
  float2 c = make_float2(0.0f, 0.0f);
  if (xl || xr || yb || yt) c = d2p[n];
  const float2 vE = xr ? c : d2p[n + 1];
  const float2 vW = xl ? c : d2p[n - 1];
  const float2 vN = yt ? c : d2p[n + P.px];
  const float2 vS = yb ? c : d2p[n - P.px];
  wall_ghosts(c, vE, vW, vN, vS, xl, xr, yb, yt, gr);
}

// One node of one time step (the whole hot path for that node).
template <bool ODD, class S, class I, int NL = 3>
__device__ __forceinline__ void step_node(const StepParams& P, typename S::T* __restrict__ pop,
                                          const float2* __restrict__ d2p, float2* __restrict__ d2c,
                                          float* __restrict__ d5, int x, int y) {
  float f[9], p[9], g[9], g2[NL == 4 ? 9 : 1];
  load_node<ODD, S, I, NL>(P, pop, d5, x, y, f, p, g, g2);

  // S4: central differences of the previous step's (phi, theta); zero-flux
  // mirror ghosts for phi on all walls and for theta on the adiabatic walls,
  // linear ghosts 2 theta_w - theta through the isothermal walls.
  const long long n = (long long)y * P.px + x;
  const bool xl = x == 0, xr = x == P.nx - 1, yb = y == 0, yt = y == P.ny - 1;
  float2 c = make_float2(0.0f, 0.0f);
  if (xl || xr || yb || yt) c = d2p[n];
  const float2 vE = xr ? c : d2p[n + 1];
  const float2 vW = xl ? c : d2p[n - 1];
  const float2 vN = yt ? c : d2p[n + P.px];
  const float2 vS = yb ? c : d2p[n - P.px];
  const float thE = xr ? (-1.0f - c.y) : vE.y;
  const float thW = xl ? (1.0f - c.y) : vW.y;
  const float gphix = 0.5f * (vE.x - vW.x), gphiy = 0.5f * (vN.x - vS.x);
  const float gthx = 0.5f * (thE - thW), gthy = 0.5f * (vN.y - vS.y);

  const float2 keep = node_update<NL>(P, f, p, g, gphix, gphiy, gthx, gthy, g2);
  store_node<ODD, S, I, NL>(P, pop, d5, x, y, f, p, g, g2);
  d2c[n] = keep;
}

template <bool ODD, class S, class I, int NL>
__global__ __launch_bounds__(256) void k_step(StepParams P,
                                              typename S::T* __restrict__ pop,
                                              const float2* __restrict__ d2p,
                                              float2* __restrict__ d2c,
                                              float* __restrict__ d5,
                                              int tiles_x) {
  const unsigned t = xcd_tile(blockIdx.x, gridDim.x);
  const int x = (int)(t % (unsigned)tiles_x) * blockDim.x + threadIdx.x;
  const int y = (int)(t / (unsigned)tiles_x) * blockDim.y + threadIdx.y;
  if (x >= P.nx || y >= P.ny) return;
  step_node<ODD, S, I, NL>(P, pop, d2p, d2c, d5, x, y);
}

// ---- two time steps per launch ---------------------------------------------
// k_step2 runs an even step t and the odd step t + 1 in one pass, reading the
// populations at t (A-A layout of an even step) from one array and writing
// those at t + 2 (same layout) to a second one, so a step needs half the
// algorithmic bytes of k_step (the halo rows that neighbouring bands read
// again add about a third).  The in-place pattern cannot be used here: the
// workgroups overlap by a halo and would overwrite what their neighbours
// still read.
//
// One wave owns a strip of kStrip2 columns and a band of rows.  Its 64 lanes
// hold the strip and one halo column on each side.  It sweeps the band
// upwards, one row r per iteration:
//   stage A  the even step on row r (all 64 lanes): load the node's own slots,
//            lag gradients of step t - 1, node update; the post-collision
//            values stay in registers;
//   pull     each value moves to the node it streams to: across lanes by one
//            shuffle (x), across rows by being carried to a later iteration
//            (y); what row r sends down (e_y = -1) is consumed now, what it
//            sends along (e_y = 0) in the next iteration, what it sends up
//            (e_y = +1) in the one after;
//   stage B  the odd step on row q = r - 1 of the strip: the pulled values
//            with the wall rules (Eqs 34-36) that the in-place odd load
//            applies, gradients from stage A's lag fields, node update, and
//            the store of the in-place odd step into the second array.
// Rows outside the band are computed by stage A as halo (one row below, one
// above), never stored.
constexpr int kStrip2 = 62;

// Dispatch order of the bands of a two-step launch.  Each XCD takes the
// band rows of its range in order, so band b + 1 of a strip would start
// about one row iteration after band b: the halo rows the two share are
// then read an iteration or two apart, by which time the XCD's L2 has
// streamed past them.  Within windows of mix x kBandWindow band rows, band
// i of the window is dispatched at slot (i % kBandWindow) * mix + i /
// kBandWindow, so neighbouring bands start mix slots apart and read their
// shared rows at about the same time.  A bijection of the band indices
// (the tail beyond the last whole window keeps its order); the tiles of a
// launch are independent, so the results do not depend on it.
constexpr int kBandWindow = 16;
__device__ __forceinline__ int band_of_tile(int slot, int segs, int mix) {
  const int w = mix * kBandWindow;
  if (mix <= 1 || slot >= segs / w * w) return slot;
  const int i = slot % w;
  return slot - i + (i % mix) * kBandWindow + i / mix;
}

// the 3 directions of each pull group, per lattice: up (e_y = +1), along
// (e_y = 0), down (e_y = -1)
__device__ __forceinline__ float pull_x(float v, int i) {
  // direction i at x comes from x - e_x(i): the lane below or above
  if (ex(i) == 1) return __shfl_up(v, 1, 64);
  if (ex(i) == -1) return __shfl_down(v, 1, 64);
  return v;
}

// One tile (strip, band segment seg) of one cavity, by one 64-lane wave.
template <class S, class I>
__device__ __forceinline__ void step2_tile(const StepParams& P, const typename S::T* __restrict__ popA,
                                           typename S::T* __restrict__ popB,
                                           const float2* __restrict__ d2p, float2* __restrict__ d2o,
                                           int strip, int seg, int band) {
  constexpr int UP[3] = {2, 5, 6}, AL[3] = {0, 1, 3}, DN[3] = {4, 7, 8};
  // What a row sends up waits two iterations: a ring of three rows in LDS,
  // one column per lane (each lane reads back only what it wrote).  The
  // x-wall lanes keep their own values for the diagonal unknowns of the odd
  // step in a two-row ring (left and right wall).
  __shared__ float s_up[3][9][64];
  __shared__ float s_xw[2][2][6];
  const int lane = (int)threadIdx.x;
  const int nx = P.nx, ny = P.ny;
  const int x = strip * kStrip2 - 1 + lane;
  const int xs = min(max(x, 0), nx - 1);  // halo lanes outside the cavity repeat the edge
  const bool xl = x == 0, xr = x == nx - 1;
  const int side = xl ? 0 : 1;
  const bool mine = lane >= 1 && lane <= kStrip2 && x < nx;
  const int y0 = seg * band, y1 = min(y0 + band, ny);
  const int ra = max(y0 - 1, 0);
  auto ring = [](int row) { return (row + 3) % 3; };  // rows >= -1

  float M[9];  // along values for row r - 1 (lattice l, slot k at [3 l + k])
  float2 dq = make_float2(0.0f, 0.0f), dqm = dq;  // lag field of step t at rows r - 1, r - 2
#pragma unroll
  for (int k = 0; k < 9; ++k) M[k] = 0.0f;

  // The loads of a row are issued in the iteration before (after its stage
  // A, before its stage B): a wave's loads and stores share one in-order
  // completion counter, so loads issued after the odd step's stores would
  // also wait for those stores.
  const int rlast = min(y1, ny - 1);  // last row of stage A
  float PF[3][9];
  load_node<false, S, I>(P, popA, nullptr, xs, ra, PF[0], PF[1], PF[2]);
  // Lag field of step t - 1 in the lane's column: rows r - 1, r and r + 1
  // carried from one iteration to the next, row r + 2 in flight; the x
  // neighbours come from the adjacent lanes, and the two lanes at the ends
  // of the wave load their outer neighbour (row r, in flight: row r + 1).
  const int xo = min(max(lane == 0 ? xs - 1 : (lane == 63 ? xs + 1 : xs), 0), nx - 1);
  auto lag = [&](int row, int col) { return d2p[(long long)min(row, ny - 1) * P.px + col]; };
  float2 Lm = lag(max(ra - 1, 0), xs), L0 = lag(ra, xs), Lp = lag(ra + 1, xs), Lo = lag(ra, xo);
  float2 Lpp = Lp, Lon = Lo;

  for (int r = ra; r <= y1; ++r) {
    const bool has_a = r < ny;
    float ALn[9], DNn[9];  // what row r sends along and down
    float2 dr = dq;
    {
      float A[3][9] = {};  // stage A: post-collision values of row r (f, p, g)
      if (has_a) {
#pragma unroll
        for (int l = 0; l < 3; ++l)
#pragma unroll
          for (int i = 0; i < 9; ++i) A[l][i] = PF[l][i];
        const float2 sE = make_float2(__shfl_down(L0.x, 1, 64), __shfl_down(L0.y, 1, 64));
        const float2 sW = make_float2(__shfl_up(L0.x, 1, 64), __shfl_up(L0.y, 1, 64));
        float4 gr;
        wall_ghosts(L0, lane == 63 ? Lo : sE, lane == 0 ? Lo : sW, Lp, Lm, xs == 0, xs == nx - 1, r == 0,
                    r == ny - 1, gr);
        dr = node_update<3>(P, A[0], A[1], A[2], gr.x, gr.y, gr.z, gr.w);
        // the next row's loads: after the stage-A update (whose first use
        // of this row's values waits for them), overlapping stage B
        if (r < rlast) {
          load_node<false, S, I>(P, popA, nullptr, xs, r + 1, PF[0], PF[1], PF[2]);
          Lpp = lag(r + 2, xs);
          Lon = lag(r + 1, xo);
        }
      }
      // pull across lanes (whole wave, uniform control flow)
      float UPn[9];
#pragma unroll
      for (int l = 0; l < 3; ++l)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          UPn[3 * l + k] = pull_x(A[l][UP[k]], UP[k]);
          ALn[3 * l + k] = pull_x(A[l][AL[k]], AL[k]);
          DNn[3 * l + k] = pull_x(A[l][DN[k]], DN[k]);
        }
      if (has_a) {
        // x walls, along directions: E at the left wall, W at the right
        // wall (bounce-back for f and p, anti-bounce-back for g, Eqs 34-35)
        if (xl) {
          ALn[1] = A[0][3];
          ALn[4] = A[1][3];
          ALn[7] = wgt(1) - A[2][3];
        }
        if (xr) {
          ALn[2] = A[0][1];
          ALn[5] = A[1][1];
          ALn[8] = -wgt(3) - A[2][1];
        }
        // x-wall lanes keep their own values for the diagonal unknowns of
        // the odd step on this row: (up, down) = (NE, SE) <- (SW, NW) on the
        // left, (NW, SW) <- (SE, NE) on the right
        if (xl || xr) {
#pragma unroll
          for (int l = 0; l < 3; ++l) {
            s_xw[r & 1][side][2 * l] = xl ? A[l][7] : A[l][8];
            s_xw[r & 1][side][2 * l + 1] = xl ? A[l][6] : A[l][5];
          }
        }
        if (r == 0) {
          // bottom wall row: its up unknowns are bounce-back of its own down
          // values (f, p) and, for g, what row 0 streams into row 1 (copy of
          // the adiabatic wall, Eq 36); corners are set in the odd step
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            s_up[ring(-1)][k][lane] = A[0][DN[k]];
            s_up[ring(-1)][3 + k][lane] = A[1][DN[k]];
            s_up[ring(-1)][6 + k][lane] = UPn[6 + k];
          }
        }
        if (r == ny - 1) {
          // top wall row: its down unknowns likewise, kept in its own slot
          // of the ring (nothing streams above the top row)
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            UPn[k] = A[0][UP[k]];
            UPn[3 + k] = A[1][UP[k]];
            UPn[6 + k] = DNn[6 + k];
          }
          // corners of g: the copy of row ny - 2 after its x-wall rule
          if (xl) UPn[8] = wgt(8) - s_xw[(r - 1) & 1][0][5];
          if (xr) UPn[7] = -wgt(7) - s_xw[(r - 1) & 1][1][5];
        }
#pragma unroll
        for (int k = 0; k < 9; ++k) s_up[ring(r)][k][lane] = UPn[k];
      }
    }
    const float2 dE = make_float2(__shfl_down(dq.x, 1, 64), __shfl_down(dq.y, 1, 64));
    const float2 dW = make_float2(__shfl_up(dq.x, 1, 64), __shfl_up(dq.y, 1, 64));

    // stage B: the odd step on row q
    const int q = r - 1;
    if (q >= y0) {
      float G[3][9];
#pragma unroll
      for (int l = 0; l < 3; ++l)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          G[l][UP[k]] = s_up[ring(r - 2)][3 * l + k][lane];
          G[l][AL[k]] = M[3 * l + k];
          G[l][DN[k]] = has_a ? DNn[3 * l + k] : s_up[ring(r - 1)][3 * l + k][lane];
        }
      // x walls, diagonal directions
      if (xl || xr) {
        const float* w = s_xw[q & 1][side];
        // g: anti-bounce-back, except where the link also crosses a y wall
        // (bottom row: the copy of row 1 after its x-wall rule; top row: set
        // with the top row's down values)
        const float gup = q > 0 ? w[4] : s_xw[r & 1][side][4];
        if (xl) {
          G[0][5] = w[0];
          G[0][8] = w[1];
          G[1][5] = w[2];
          G[1][8] = w[3];
          G[2][5] = wgt(5) - gup;
          if (q < ny - 1) G[2][8] = wgt(8) - w[5];
        } else {
          G[0][6] = w[0];
          G[0][7] = w[1];
          G[1][6] = w[2];
          G[1][7] = w[3];
          G[2][6] = -wgt(6) - gup;
          if (q < ny - 1) G[2][7] = -wgt(7) - w[5];
        }
      }
      float4 gr;
      wall_ghosts(dq, dE, dW, dr, dqm, xl, xr, q == 0, q == ny - 1, gr);
      const float2 keep = node_update<3>(P, G[0], G[1], G[2], gr.x, gr.y, gr.z, gr.w);
      if (mine) {
        store_node<true, S, I>(P, popB, nullptr, x, q, G[0], G[1], G[2]);
        d2o[(long long)q * P.px + x] = keep;
      }
    }
    if (!has_a) break;
#pragma unroll
    for (int k = 0; k < 9; ++k) M[k] = ALn[k];
    dqm = dq;
    dq = dr;
    Lm = L0;
    L0 = Lp;
    Lp = Lpp;
    Lo = Lon;
  }
}

template <class S, class I>
__global__ __launch_bounds__(64) void k_step2(StepParams P, const typename S::T* __restrict__ popA,
                                              typename S::T* __restrict__ popB,
                                              const float2* __restrict__ d2p, float2* __restrict__ d2o,
                                              int strips, int band, int mix) {
  const unsigned tile = xcd_tile(blockIdx.x, gridDim.x);
  step2_tile<S, I>(P, popA, popB, d2p, d2o, (int)(tile % (unsigned)strips),
                band_of_tile((int)(tile / (unsigned)strips), (P.ny + band - 1) / band, mix), band);
}

// Batched sweep: one launch per time step updates every active cavity of a
// batch of uneven cavities.  Each entry of the tile table names a cavity and
// one 256-node tile of it (shape bx x by chosen per cavity); workgroup b
// takes entries b, b + G, b + 2G, ... (the host sizes G to the table, so one
// entry each).  The table is laid out so that the entries of one XCD are
// neighbours in space.  The entry count is read from device memory, so a captured
// graph of this launch stays valid when cavities drop out of the table.
//
// Batches with two steps per launch keep two population copies per cavity
// and a second table of (strip, band) tiles for k_step2_batch.  Every launch
// of two steps swaps the roles of the copies and of the two lag fields for
// all active cavities at once; the descriptors hold the roles at the time
// they were written and each launch takes flip, the number of two-step
// launches since then modulo 2.
struct CavDesc {
  StepParams P;
  void* pop[2];  // current and other population copy (the same without a second copy)
  float2* d2[2];
  float* d5;
  int tiles_x, bx, by, strips2, band2, pad;
};

template <bool ODD, class S, class I>
__global__ __launch_bounds__(256) void k_step_batch(const CavDesc* __restrict__ cavs,
                                                    const int2* __restrict__ tiles,
                                                    const int* __restrict__ ntiles_p, int flip) {
  const int ntiles = *ntiles_p;
  for (int k = blockIdx.x; k < ntiles; k += gridDim.x) {
    const int2 tr = tiles[k];
    if (tr.x < 0) continue;  // padding entry
    const CavDesc& C = cavs[tr.x];
    const int bx = C.bx;
    const int x = (tr.y % C.tiles_x) * bx + (int)threadIdx.x % bx;
    const int y = (tr.y / C.tiles_x) * C.by + (int)threadIdx.x / bx;
    if (x < C.P.nx && y < C.P.ny)
      step_node<ODD, S, I>(C.P, reinterpret_cast<typename S::T*>(C.pop[flip]), C.d2[(ODD ? 0 : 1) ^ flip],
                           C.d2[(ODD ? 1 : 0) ^ flip], C.d5, x, y);
  }
}

// Two steps per launch over a batch: one 64-lane workgroup per entry of the
// (strip, band) table, each running the tile of k_step2.
template <class S>
__global__ __launch_bounds__(64) void k_step2_batch(const CavDesc* __restrict__ cavs,
                                                    const int2* __restrict__ tiles,
                                                    const int* __restrict__ ntiles_p, int flip) {
  if ((int)blockIdx.x >= *ntiles_p) return;
  const int2 tr = tiles[blockIdx.x];
  if (tr.x < 0) return;  // padding entry
  const CavDesc& C = cavs[tr.x];
  using T = typename S::T;
  step2_tile<S, uint32_t>(C.P, reinterpret_cast<const T*>(C.pop[flip]), reinterpret_cast<T*>(C.pop[flip ^ 1]),
                C.d2[1 ^ flip], C.d2[flip], tr.y % C.strips2, tr.y / C.strips2, C.band2);
}

// Many small cavities: one 1024-thread workgroup owns a whole cavity (at
// most kPerCavNodes nodes) and runs `steps` steps of it, an even number from
// an even step, with a workgroup barrier between the steps.  The launch
// overhead of one launch per step goes, and the cavity's arrays stay in the
// caches of one XCD; a cavity then has one compute unit, so this pays only
// with about as many cavities as compute units.  list: the active
// cavities.  The node updates are those of k_step_batch (bitwise equal).
constexpr int kPerCavThreads = 1024;
constexpr int kPerCavNodes = 128 * 128;
template <class SE, class SO, class I>
__global__ __launch_bounds__(kPerCavThreads) void k_step_cavity(const CavDesc* __restrict__ cavs,
                                                                const int* __restrict__ list, int steps) {
  const CavDesc& C = cavs[list[blockIdx.x]];
  auto* pop = reinterpret_cast<typename SE::T*>(C.pop[0]);  // one copy: no second role
  const int nx = C.P.nx, nn = C.P.nx * C.P.ny;
  for (int s = 0; s < steps; s += 2) {
    for (int n = (int)threadIdx.x; n < nn; n += kPerCavThreads)
      step_node<false, SE, I>(C.P, pop, C.d2[1], C.d2[0], C.d5, n % nx, n / nx);
    __syncthreads();
    for (int n = (int)threadIdx.x; n < nn; n += kPerCavThreads)
      step_node<true, SO, I>(C.P, pop, C.d2[0], C.d2[1], C.d5, n % nx, n / nx);
    __syncthreads();
  }
}

// Block-wide FP64 sum; wave64 shuffles then one LDS slot per wave.
__device__ double block_sum(double v, double* lds) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) lds[wid] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int w = 0; w < nw; ++w) r += lds[w];
  }
  return r;
}

// Temperatures at a node in FP64: fluid (first thermal lattice), particles
// (second thermal lattice, or the same one) and the suspension (Eq 33 over
// the two lattices with volume fractions 1 - phi, phi and heat capacities
// per volume in the ratio 1 : 1 + crc).
template <int NL>
__device__ __forceinline__ double3 node_thetas(const float g[9], const float g2[9], double phi, double crc) {
  double tf = 0.0;
  for (int i = 0; i < 9; ++i) tf += (double)g[i];
  if constexpr (NL == 3) {
    return make_double3(tf, tf, tf);
  } else {
    double tp = 0.0;
    for (int i = 0; i < 9; ++i) tp += (double)g2[i];
    const double pc = phi > 0.0 ? phi : 0.0;
    return make_double3(tf, tp, (tf + pc * ((1.0 + crc) * tp - tf)) / (1.0 + crc * pc));
  }
}

// Wall-Nusselt numbers of one cavity by one workgroup (FP64).
template <bool ODD, class S, class I, int NL>
__device__ __forceinline__ void nusselt_body(const StepParams& P, const typename S::T* __restrict__ pop,
                                             const float* __restrict__ d5, double rho_p_ref, double R,
                                             double Ck, double* __restrict__ out) {
  __shared__ double lds[4];
  const int nx = P.nx, ny = P.ny;
  double sh = 0.0, sc = 0.0, sk = 0.0, bad = 0.0;
  for (int y = threadIdx.x; y < ny; y += blockDim.x) {
    const int xs[4] = {0, 1, nx - 2, nx - 1};
    double th[4];
    double rp0 = rho_p_ref;
    for (int q = 0; q < 4; ++q) {
      float f[9], p[9], g[9], g2[NL == 4 ? 9 : 1];
      load_node<ODD, S, I, NL>(P, pop, d5, xs[q], y, f, p, g, g2);
      double rp = rho_p_ref;
      for (int i = 0; i < 9; ++i) rp += (double)p[i];
      th[q] = node_thetas<NL>(g, g2, rp / R, (double)P.crc).z;
      if (q == 0) rp0 = rp;
    }
    double phi = rp0 / R;
    if (phi < 0.0) phi = 0.0;
    const double rk = 1.0 + Ck * pow(phi, 0.764);
    const double gh = -(double)nx * (9.0 * th[0] - th[1] - 4.0) / 3.0;
    const double gc = (double)nx * (9.0 * th[3] - th[2] + 4.0) / 3.0;
    sh += gh;
    sc += gc;
    sk += rk * gh;
    if (!isfinite(gh) || !isfinite(gc)) bad = 1.0;
  }
  sh = block_sum(sh, lds);
  sc = block_sum(sc, lds);
  sk = block_sum(sk, lds);
  bad = block_sum(bad, lds);
  if (threadIdx.x == 0) {
    out[0] = sh / ny;
    out[1] = sc / ny;
    out[2] = sk / ny;
    out[3] = bad;
  }
}

template <bool ODD, class S, class I, int NL>
__global__ __launch_bounds__(256) void k_nusselt(StepParams P,
                                                 const typename S::T* __restrict__ pop,
                                                 const float* __restrict__ d5,
                                                 double rho_p_ref, double R,
                                                 double Ck,
                                                 double* __restrict__ out) {
  nusselt_body<ODD, S, I, NL>(P, pop, d5, rho_p_ref, R, Ck, out);
}

// Per-block partial sums of |u - u_ref|^2, |u|^2, (theta - theta_ref)^2,
// theta^2 and a non-finite count; the snapshot is replaced by the state.
template <bool ODD, class S, class I, int NL>
__device__ __forceinline__ void residual_block(const StepParams& P, const typename S::T* __restrict__ pop,
                                               const float* __restrict__ d5, double rho_f_ref,
                                               double rho_p_ref, double* __restrict__ snap,
                                               double* __restrict__ partial, int block) {
  __shared__ double lds[4];
  const long long nn = (long long)P.nx * P.ny;
  const long long k = (long long)block * blockDim.x + threadIdx.x;
  double du = 0.0, un = 0.0, dt = 0.0, tn = 0.0, bad = 0.0;
  if (k < nn) {
    const int x = (int)(k % P.nx), y = (int)(k / P.nx);
    float f[9], p[9], g[9], g2[NL == 4 ? 9 : 1];
    load_node<ODD, S, I, NL>(P, pop, d5, x, y, f, p, g, g2);
    double rf = rho_f_ref, rp = rho_p_ref, jx = 0.0, jy = 0.0;
    for (int i = 0; i < 9; ++i) {
      rf += (double)f[i];
      rp += (double)p[i];
      jx += (double)ex(i) * ((double)f[i] + (double)p[i]);
      jy += (double)ey(i) * ((double)f[i] + (double)p[i]);
    }
    const double th = node_thetas<NL>(g, g2, rp * (double)P.invR, (double)P.crc).z;
    const double ux = jx / (rf + rp), uy = jy / (rf + rp);
    const double ox = snap[k], oy = snap[nn + k], ot = snap[2 * nn + k];
    du = (ux - ox) * (ux - ox) + (uy - oy) * (uy - oy);
    un = ux * ux + uy * uy;
    dt = (th - ot) * (th - ot);
    tn = th * th;
    if (!isfinite(ux) || !isfinite(uy) || !isfinite(th)) bad = 1.0;
    snap[k] = ux;
    snap[nn + k] = uy;
    snap[2 * nn + k] = th;
  }
  du = block_sum(du, lds);
  un = block_sum(un, lds);
  dt = block_sum(dt, lds);
  tn = block_sum(tn, lds);
  bad = block_sum(bad, lds);
  if (threadIdx.x == 0) {
    double* o = partial + 5 * (long long)block;
    o[0] = du; o[1] = un; o[2] = dt; o[3] = tn; o[4] = bad;
  }
}

template <bool ODD, class S, class I, int NL>
__global__ __launch_bounds__(256) void k_residual(StepParams P,
                                                  const typename S::T* __restrict__ pop,
                                                  const float* __restrict__ d5,
                                                  double rho_f_ref, double rho_p_ref,
                                                  double* __restrict__ snap,
                                                  double* __restrict__ partial) {
  residual_block<ODD, S, I, NL>(P, pop, d5, rho_f_ref, rho_p_ref, snap, partial, (int)blockIdx.x);
}

// Fixed-order sum of the per-block partials (deterministic).
__device__ __forceinline__ void sum_partials_body(const double* __restrict__ partial, int nblocks,
                                                  double* __restrict__ out) {
  __shared__ double lds[4];
  for (int q = 0; q < 5; ++q) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) s += partial[5 * (long long)b + q];
    s = block_sum(s, lds);
    if (threadIdx.x == 0) out[q] = s;
  }
}

__global__ __launch_bounds__(256) void k_sum_partials(const double* __restrict__ partial,
                                                      int nblocks,
                                                      double* __restrict__ out) {
  sum_partials_body(partial, nblocks, out);
}

// The same fixed-order sum, finished on the device: out[0] = residual of
// the mixture velocity, out[1] = residual of theta (the host formulas of
// mclbm_residual, in FP64), out[2] = 1 if any node was non-finite, else 0.
__global__ __launch_bounds__(256) void k_sum_partials_finish(const double* __restrict__ partial,
                                                             int nblocks,
                                                             double* __restrict__ out) {
  __shared__ double sums[5];
  sum_partials_body(partial, nblocks, sums);
  __syncthreads();
  if (threadIdx.x == 0) {
    const double du = sums[0], un = sums[1], dt = sums[2], tn = sums[3];
    out[0] = un > 0.0 ? sqrt(du / un) : (du > 0.0 ? (double)INFINITY : 0.0);
    out[1] = tn > 0.0 ? sqrt(dt / tn) : (dt > 0.0 ? (double)INFINITY : 0.0);
    out[2] = sums[4] != 0.0 ? 1.0 : 0.0;
  }
}

// The reductions of every active cavity of a batch (all at one step
// parity, current copy C.pop[flip]) in three launches: the Nusselt numbers
// and the summed partials one workgroup per cavity, the residual's partials
// one workgroup per (cavity, block) entry.  Results go to out[16 j ..]
// for the j-th cavity of the list: Nu at 0-3, the residual sums at 4-8.
struct RedDesc {
  double* snap;
  double* part;
  double rho_f_ref, rho_p_ref, R, Ck;
  int red_blocks, pad;
};

template <bool ODD, class S, class I>
__global__ __launch_bounds__(256) void k_nusselt_batch(const CavDesc* __restrict__ cavs,
                                                       const RedDesc* __restrict__ red,
                                                       const int* __restrict__ list, int flip,
                                                       double* __restrict__ out) {
  const int m = list[blockIdx.x];
  const CavDesc& C = cavs[m];
  nusselt_body<ODD, S, I, 3>(C.P, reinterpret_cast<const typename S::T*>(C.pop[flip]), C.d5,
                             red[m].rho_p_ref, red[m].R, red[m].Ck, out + 16 * (long long)blockIdx.x);
}

template <bool ODD, class S, class I>
__global__ __launch_bounds__(256) void k_residual_batch(const CavDesc* __restrict__ cavs,
                                                        const RedDesc* __restrict__ red,
                                                        const int2* __restrict__ tiles, int flip) {
  const int2 e = tiles[blockIdx.x];
  const CavDesc& C = cavs[e.x];
  residual_block<ODD, S, I, 3>(C.P, reinterpret_cast<const typename S::T*>(C.pop[flip]), C.d5,
                               red[e.x].rho_f_ref, red[e.x].rho_p_ref, red[e.x].snap, red[e.x].part, e.y);
}

__global__ __launch_bounds__(256) void k_sum_partials_batch(const RedDesc* __restrict__ red,
                                                            const int* __restrict__ list,
                                                            double* __restrict__ out) {
  const int m = list[blockIdx.x];
  sum_partials_body(red[m].part, red[m].red_blocks, out + 16 * (long long)blockIdx.x + 4);
}

// Warm start: bilinear samples of channel-last fields (sy x sx x nc) at
// the lattice nodes, cell-centred on both grids, in FP64.
struct FieldMap {
  const float* F;
  int sx, sy, nc;
  double a[5], b[5];
};

__device__ __forceinline__ void field_axis(int i, int n_dst, int n_src, int& i0, int& i1, double& w) {
  double s = ((double)i + 0.5) * (double)n_src / (double)n_dst - 0.5;
  s = fmin(fmax(s, 0.0), (double)(n_src - 1));
  i0 = (int)floor(s);
  i1 = min(i0 + 1, n_src - 1);
  w = s - (double)i0;
}

struct FieldPoint {
  int x0, x1, y0, y1;
  double wx, wy;
};

__device__ __forceinline__ FieldPoint field_point(const FieldMap& M, int x, int y, int nx, int ny) {
  FieldPoint q;
  field_axis(x, nx, M.sx, q.x0, q.x1, q.wx);
  field_axis(y, ny, M.sy, q.y0, q.y1, q.wy);
  return q;
}

__device__ __forceinline__ double field_sample(const FieldMap& M, int c, const FieldPoint& q) {
  auto v = [&](int yy, int xx) {
    return M.a[c] * (double)M.F[((long long)yy * M.sx + xx) * M.nc + c] + M.b[c];
  };
  return (1.0 - q.wy) * ((1.0 - q.wx) * v(q.y0, q.x0) + q.wx * v(q.y0, q.x1)) +
         q.wy * ((1.0 - q.wx) * v(q.y1, q.x0) + q.wx * v(q.y1, q.x1));
}

// Per-block sums of the clipped phi samples (slot 0 of 5 per block) and of
// the fluid-density deviation samples (slot 1; 0 without that channel).
__global__ __launch_bounds__(256) void k_load_sums(FieldMap M, int nx, int ny, double* __restrict__ partial) {
  __shared__ double lds[4];
  const long long nn = (long long)nx * ny;
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  double s = 0.0, r = 0.0;
  if (k < nn) {
    const FieldPoint q = field_point(M, (int)(k % nx), (int)(k / nx), nx, ny);
    s = fmax(field_sample(M, 3, q), 0.0);
    if (M.nc > 4) r = field_sample(M, 4, q);
  }
  s = block_sum(s, lds);
  r = block_sum(r, lds);
  if (threadIdx.x == 0) {
    double* o = partial + 5 * (long long)blockIdx.x;
    o[0] = s; o[1] = r; o[2] = 0.0; o[3] = 0.0; o[4] = 0.0;
  }
}

// Constants of the warm start in FP64.
struct LoadConst {
  double inventory, rho_f0, R, tau_f, alpha3, Ck, crc_m1;
};

// Gradient along one axis of sampled values at lattice nodes: central
// differences inside, one-sided at the first and last node (so fields
// without gradients give none at the walls either).
__device__ __forceinline__ double node_diff(double lo, double mid, double hi, bool first, bool last) {
  if (first) return hi - mid;
  if (last) return mid - lo;
  return 0.5 * (hi - lo);
}

// Populations of the sampled fields: the equilibria (Eqs 26-27) plus the
// first-order non-equilibrium parts of the Chapman-Enskog expansion of the
// BGK lattices (Eqs 18-19), the viscous stress of the fluid lattice,
// -3 tau_f W_i rho_f (e_i e_i - I/3) : grad u, and the conducted heat flux of
// the temperature lattice, -tau_theta W_i e_i . grad theta (tau_theta of
// Eq 24 at the node's phi); the particle lattice takes its equilibrium.
// phi is rescaled to the cold-start inventory, the fluid partial density
// is that of the cold start plus the sampled deviation less its lattice
// mean (so both phases keep their cold-start mass).  Then the lag field of
// the first step from the stored state, as at a cold start.
template <class S>
__global__ __launch_bounds__(256) void k_load_fields(StepParams P, FieldMap M, LoadConst K,
                                                     typename S::T* __restrict__ pop,
                                                     const double* __restrict__ sums,
                                                     float2* __restrict__ d2prev) {
  const long long nn = (long long)P.nx * P.ny;
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nn) return;
  const int x = (int)(k % P.nx), y = (int)(k / P.nx);
  const FieldPoint q = field_point(M, x, y, P.nx, P.ny);
  const double ux = field_sample(M, 0, q);
  const double uy = field_sample(M, 1, q);
  const double th = field_sample(M, 2, q);
  // the u and theta samples at the four neighbours
  const bool xf = x == 0, xl = x == P.nx - 1, yf = y == 0, yl = y == P.ny - 1;
  double nb[4][3];  // E, W, N, S
  const int nxs[4] = {xl ? x : x + 1, xf ? x : x - 1, x, x};
  const int nys[4] = {y, y, yl ? y : y + 1, yf ? y : y - 1};
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    const FieldPoint r = field_point(M, nxs[d], nys[d], P.nx, P.ny);
#pragma unroll
    for (int c = 0; c < 3; ++c) nb[d][c] = field_sample(M, c, r);
  }
  const double dxux = node_diff(nb[1][0], ux, nb[0][0], xf, xl);
  const double dxuy = node_diff(nb[1][1], uy, nb[0][1], xf, xl);
  const double dxth = node_diff(nb[1][2], th, nb[0][2], xf, xl);
  const double dyux = node_diff(nb[3][0], ux, nb[2][0], yf, yl);
  const double dyuy = node_diff(nb[3][1], uy, nb[2][1], yf, yl);
  const double dyth = node_diff(nb[3][2], th, nb[2][2], yf, yl);

  const double total = sums[0];
  double phi = fmax(field_sample(M, 3, q), 0.0);
  phi = total > 0.0 ? phi * (K.inventory / total) : K.inventory / (double)nn;
  double rf = K.rho_f0;
  if (M.nc > 4) rf += field_sample(M, 4, q) - sums[1] / (double)nn;
  const double rp = K.R * phi;
  const double tau_th = K.alpha3 * (1.0 + K.Ck * pow(phi, 0.764)) / (1.0 + phi * K.crc_m1) + 0.5;
  const double rf_ref = (double)P.rho_f_ref, rp_ref = (double)P.rho_p_ref;
  const double uu = ux * ux + uy * uy;
  const double shear = dxuy + dyux;
  const long long n = (long long)y * P.px + x;
  float f[9], p[9], g[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const double exi = (double)ex(i), eyi = (double)ey(i);
    const double eu = exi * ux + eyi * uy;
    const double shape = 3.0 * eu + 4.5 * eu * eu - 1.5 * uu;
    const double w = wgt_d(i);
    const double qgu = (exi * exi - 1.0 / 3.0) * dxux + (eyi * eyi - 1.0 / 3.0) * dyuy + exi * eyi * shear;
    const double fneq = -3.0 * K.tau_f * w * rf * qgu;
    const double gneq = -tau_th * w * (exi * dxth + eyi * dyth);
    S::st(pop + P.plane * i + n, (float)(w * ((rf - rf_ref) + rf * shape) + fneq), P.scale[0]);
    S::st(pop + P.plane * (9 + i) + n, (float)(w * ((rp - rp_ref) + rp * shape)), P.scale[1]);
    S::st(pop + P.plane * (18 + i) + n, (float)(w * th * (1.0 + shape) + gneq), P.scale[2]);
  }
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    f[i] = S::ld(pop + P.plane * i + n, P.inv_scale[0]);
    p[i] = S::ld(pop + P.plane * (9 + i) + n, P.inv_scale[1]);
    g[i] = S::ld(pop + P.plane * (18 + i) + n, P.inv_scale[2]);
  }
  const NodeMoments m = moments(f, p, g);
  d2prev[n] = make_float2(m.drp * P.invR, m.th);
}

template <bool ODD, class S, class I, int NL>
__global__ __launch_bounds__(256) void k_export(StepParams P,
                                                const typename S::T* __restrict__ pop,
                                                const float* __restrict__ d5,
                                                double rho_f_ref, double rho_p_ref,
                                                double invR, unsigned mask,
                                                double* __restrict__ out) {
  const long long nn = (long long)P.nx * P.ny;
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nn) return;
  const int x = (int)(k % P.nx), y = (int)(k / P.nx);
  float f[9], p[9], g[9], g2[NL == 4 ? 9 : 1];
  load_node<ODD, S, I, NL>(P, pop, d5, x, y, f, p, g, g2);
  double rf = rho_f_ref, rp = rho_p_ref, jxf = 0, jyf = 0, jxp = 0, jyp = 0;
  for (int i = 0; i < 9; ++i) {
    rf += (double)f[i];
    rp += (double)p[i];
    jxf += (double)ex(i) * (double)f[i];
    jyf += (double)ey(i) * (double)f[i];
    jxp += (double)ex(i) * (double)p[i];
    jyp += (double)ey(i) * (double)p[i];
  }
  const double3 th = node_thetas<NL>(g, g2, rp * invR, (double)P.crc);
  const double uxf = jxf / rf, uyf = jyf / rf;
  const bool empty = !(rp > 1e-12);
  const double v[MCLBM_FIELD_COUNT] = {rf, uxf, uyf, rp * invR,
                                       empty ? uxf : jxp / rp, empty ? uyf : jyp / rp, th.z,
                                       (jxf + jxp) / (rf + rp), (jyf + jyp) / (rf + rp), th.x, th.y};
  int slot = 0;
  for (int b = 0; b < MCLBM_FIELD_COUNT; ++b) {
    if ((mask >> b) & 1u) {
      out[(long long)slot * nn + k] = v[b];
      ++slot;
    }
  }
}

// Populations after streaming with the storage shift added back; q < 0
// writes all 9 NL planes, otherwise only plane q (lattice q / 9, direction
// q % 9) into out[0 .. nx*ny).
template <bool ODD, class S, class I, int NL>
__global__ __launch_bounds__(256) void k_export_pops(StepParams P,
                                                     const typename S::T* __restrict__ pop,
                                                     const float* __restrict__ d5,
                                                     double rho_f_ref, double rho_p_ref,
                                                     int q, double* __restrict__ out) {
  const long long nn = (long long)P.nx * P.ny;
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nn) return;
  const int x = (int)(k % P.nx), y = (int)(k / P.nx);
  float f[9], p[9], g[9], g2[NL == 4 ? 9 : 1];
  load_node<ODD, S, I, NL>(P, pop, d5, x, y, f, p, g, g2);
  for (int i = 0; i < 9; ++i) {
    const double w = wgt_d(i);
    const double v[4] = {(double)f[i] + w * rho_f_ref, (double)p[i] + w * rho_p_ref, (double)g[i],
                         NL == 4 ? (double)g2[NL == 4 ? i : 0] : 0.0};
    for (int l = 0; l < NL; ++l) {
      if (q < 0) out[(long long)(9 * l + i) * nn + k] = v[l];
      else if (q == 9 * l + i) out[k] = v[l];
    }
  }
}

// Streaming copy: each workgroup moves one contiguous block of 4 x 256
// 16-byte vectors, all four loads of a lane in flight before its stores,
// past the caches (the fastest of the simple forms measured on MI355X).
typedef float v4f __attribute__((ext_vector_type(4)));
constexpr int kCopyUnroll = 4;
// Fill with quiet NaN (race check of the step kernel).
__global__ __launch_bounds__(256) void k_poison(float* __restrict__ p, long long n) {
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (long long)gridDim.x * blockDim.x)
    p[k] = __builtin_nanf("");
}

// Population storage conversion between two cavities of one layout: each
// stored deviation read in the source's type and scale, written in the
// destination's (the reference state does not depend on the storage).
template <class SS, class SD>
__global__ __launch_bounds__(256) void k_convert(const typename SS::T* __restrict__ src,
                                                 typename SD::T* __restrict__ dst, long long plane,
                                                 long long n, StepParams PS, StepParams PD) {
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (long long)gridDim.x * blockDim.x) {
    const int l = min((int)(k / (9 * plane)), 2);
    SD::st(dst + k, SS::ld(src + k, PS.inv_scale[l]), PD.scale[l]);
  }
}

__global__ __launch_bounds__(256) void k_copy(v4f* __restrict__ dst,
                                              const v4f* __restrict__ src,
                                              long long n) {
  const long long base = (long long)blockIdx.x * (256 * kCopyUnroll) + threadIdx.x;
  v4f v[kCopyUnroll];
#pragma unroll
  for (int u = 0; u < kCopyUnroll; ++u) {
    const long long k = base + 256LL * u;
    if (k < n) v[u] = __builtin_nontemporal_load(src + k);
  }
#pragma unroll
  for (int u = 0; u < kCopyUnroll; ++u) {
    const long long k = base + 256LL * u;
    if (k < n) __builtin_nontemporal_store(v[u], dst + k);
  }
}

// ===========================================================================
// Host side
// ===========================================================================

namespace {

thread_local std::string g_err;

}  // namespace

namespace mclbm_host {
void set_last_error(const std::string& msg) { g_err = msg; }
}  // namespace mclbm_host

namespace {

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(MCLBM_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(expr)                                  \
  do {                                                 \
    hipError_t e_ = (expr);                            \
    if (e_ != hipSuccess) return hip_fail(e_, #expr);  \
  } while (0)

// Physical constants (SI).
constexpr double kBoltzmann = 1.380649e-23;
constexpr double kGravity = 9.81;
constexpr double kPi = 3.14159265358979323846;
// Table 1: thermophoresis C_S, C_t, C_m; Saffman K_S.
constexpr double kCs = 1.17, kCt = 2.18, kCm = 1.14, kKs = 81.2;

struct Derived {
  double v[MCLBM_D_COUNT];
};

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Layout {
  int px;
  long long plane;
  size_t off_pop, off_pop2, off_d2, off_d5, off_snap, off_part, off_res, off_stage, total;
  int red_blocks;
};

int storage_bytes(int storage) { return storage == MCLBM_FP32S ? 4 : 2; }
// lattices of a configuration: f, p and one or two thermal lattices
int lattices(const mclbm_config& c) { return c.thermal_lattices == 2 ? 4 : 3; }

// Working sets above this size stream from HBM; below it they stay in the
// 256 MB last-level (Infinity) cache, where non-temporal access hurts.
constexpr size_t kStreamingBytes = 160u << 20;

// Elements between the starts of two population planes (and of the two
// lag-field buffers): px * ny, plus kPlanePad from 2^20 nodes on.  Without
// the pad every plane of a large cavity starts at the same offset modulo a
// large power of two, so the 27 (or 54, with two copies) streams a step reads
// and writes at one node meet in the same memory channels and banks.  Pads of
// 0, 4160, 16512, 65600 and 131136 elements were timed at 1024^2, 1536^2,
// 2048^2, 3072^2 and 4096^2: 4160 was never slower than no pad (two steps
// per launch +1 % to +11 %, one step +2 %), the larger pads were faster at
// some sizes and up to 20 % slower at others.  Below 2^20 nodes, inside the
// last-level cache, the pad does not pay (512^2: 2.6 % slower).
// MCLBM_PLANE_PAD (elements, a multiple of 64, 0 to 2^20) overrides it
// (tuning knob).
constexpr long long kPlanePad = 4160;
long long plane_of(const mclbm_config& c, bool pad_planes = false) {
  const long long px = (c.nx + 63) / 64 * 64;
  long long pad = pad_planes || (long long)c.nx * c.ny >= (1LL << 20) ? kPlanePad : 0;
  if (const char* e = std::getenv("MCLBM_PLANE_PAD")) {
    const long long v = std::atoll(e);
    if (v >= 0 && v % 64 == 0 && v <= (1 << 20)) pad = v;
  }
  return px * c.ny + pad;
}

size_t pop_bytes(const mclbm_config& c, long long plane) {
  return (size_t)9 * lattices(c) * (size_t)plane * storage_bytes(c.storage);
}
size_t pop_bytes(const mclbm_config& c) { return pop_bytes(c, plane_of(c)); }

// Two time steps per launch (k_step2): one thermal lattice; population
// arrays of 2 GiB and more take 64-bit element offsets (4608^2: 32.4 GLUPS
// against 20.8 with one step per launch; at 4096^2 the 64-bit offsets cost
// 7 %).  By default for FP32 storage from 2^20 nodes and 256 columns on,
// where it was measured faster than one step per launch (1024^2 +8 %,
// 2048^2 +18 %, 4096^2 +44 % before the plane pad; slower at 512^2, and
// with 16-bit storage at every size).  The batch kernel takes 32-bit
// offsets only: batches need every member below 2 GiB of populations.
bool two_step_possible(const mclbm_config& c) { return lattices(c) == 3; }
bool two_step_batchable(const mclbm_config& c) {
  return two_step_possible(c) && pop_bytes(c) < ((size_t)1 << 31);
}
bool two_step(const mclbm_config& c, bool batch_member) {
  if (!(batch_member ? two_step_batchable(c) : two_step_possible(c))) return false;
  if (c.steps_per_launch != 0) return c.steps_per_launch == 2;
  if (batch_member) return false;  // a batch writes its own choice (member_config)
  return c.storage == MCLBM_FP32S && (long long)c.nx * c.ny >= (1LL << 20) && c.nx >= 256;
}

// Band height of the two-step kernel: 6 rows below 2^21 nodes and 3 from
// there on (of 2 to 32 rows, the fastest at 1024^2, 1536^2, 2048^2, 3072^2
// and 4096^2 with padded planes, by 1-2 % over 4 rows: more waves in flight
// outweigh the halo rows recomputed, whose loads hit in L2); MCLBM_BAND2
// sets it (tuning knob).
int band2_of(const mclbm_config& c) {
  int band = (long long)c.nx * c.ny >= (1LL << 21) ? 3 : 6;
  if (const char* e = std::getenv("MCLBM_BAND2")) {
    const int v = std::atoi(e);
    if (v >= 1 && v <= 65536) band = v;
  }
  return band;
}
int strips2_of(const mclbm_config& c) { return (c.nx + kStrip2 - 1) / kStrip2; }

// Band interleave of the two-step launch (band_of_tile): from 2^21 nodes
// on, about 150 / strips band rows (1 to 8).  Of 1 to 10 at 1536^2, 2048^2,
// 2560^2, 3072^2 and 4096^2 (25 to 67 strips) this is the fastest or
// within 1.2 % of it, +3 % to +4.5 % over dispatching the bands in order;
// below 2^21 nodes (bands of 6 rows) the bands keep their order.
// MCLBM_BANDMIX sets it (tuning knob).
int mix2_of(const mclbm_config& c) {
  int mix = 1;
  if ((long long)c.nx * c.ny >= (1LL << 21)) {
    const int strips = strips2_of(c);
    mix = std::min(8, std::max(1, (150 + strips / 2) / strips));
  }
  if (const char* e = std::getenv("MCLBM_BANDMIX")) {
    const int v = std::atoi(e);
    if (v >= 1 && v <= 64) mix = v;
  }
  return mix;
}

// pad_planes: pad the planes whatever the size (members of a batch whose
// working set streams from HBM)
Layout make_layout(const mclbm_config& c, bool batch_member = false, bool pad_planes = false) {
  Layout L{};
  L.px = (c.nx + 63) / 64 * 64;
  L.plane = plane_of(c, pad_planes);
  const long long nn = (long long)c.nx * c.ny;
  size_t off = 0;
  L.off_pop = off;
  off = align_up(off + pop_bytes(c, L.plane));
  L.off_pop2 = off;  // second copy (two steps per launch), else empty
  if (two_step(c, batch_member)) off = align_up(off + pop_bytes(c, L.plane));
  L.off_d2 = off;
  off = align_up(off + (size_t)2 * L.plane * sizeof(float2));
  L.off_d5 = off;
  off = align_up(off + (size_t)6 * (lattices(c) - 2) * L.px * sizeof(float));
  L.off_snap = off;
  off = align_up(off + (size_t)3 * nn * sizeof(double));
  L.red_blocks = (int)((nn + 255) / 256);
  L.off_part = off;
  off = align_up(off + (size_t)5 * L.red_blocks * sizeof(double));
  L.off_res = off;
  off = align_up(off + 16 * sizeof(double));
  L.off_stage = off;
  off = align_up(off + (size_t)nn * sizeof(double));
  L.total = off;
  return L;
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

int validate(const mclbm_config* c) {
  if (!c) return fail(MCLBM_EINVAL, "config is NULL");
  if (c->nx < 4 || c->ny < 4 || c->nx > 65536 || c->ny > 65536)
    return fail(MCLBM_EINVAL, "nx and ny must lie in [4, 65536]");
  if (!std::isfinite(c->Ra) || c->Ra < 0.0) return fail(MCLBM_EINVAL, "Ra must be finite and >= 0");
  if (!finite_pos(c->Pr)) return fail(MCLBM_EINVAL, "Pr must be > 0");
  if (!std::isfinite(c->phi0) || c->phi0 < 0.0 || c->phi0 > 0.1)
    return fail(MCLBM_EINVAL, "phi0 must lie in [0, 0.1]");
  if (!finite_pos(c->dp_m)) return fail(MCLBM_EINVAL, "dp_m must be > 0");
  if (!std::isfinite(c->tau_f) || (c->tau_f > 0.0 && c->tau_f <= 0.5))
    return fail(MCLBM_EINVAL, "tau_f must be > 0.5 (or <= 0 for automatic)");
  if (!finite_pos(c->dT_K) || !finite_pos(c->T0_K)) return fail(MCLBM_EINVAL, "dT_K and T0_K must be > 0");
  if (!(c->dT_K < 2.0 * c->T0_K)) return fail(MCLBM_EINVAL, "dT_K must be below 2 T0_K");
  const mclbm_material& f = c->fluid;
  const mclbm_material& p = c->particle;
  if (!finite_pos(f.rho) || !finite_pos(f.cp) || !finite_pos(f.k) || !finite_pos(f.beta) ||
      !finite_pos(f.mu) || !finite_pos(f.d_mol))
    return fail(MCLBM_EINVAL, "fluid properties must be > 0");
  if (!finite_pos(p.rho) || !finite_pos(p.cp) || !finite_pos(p.k) || !std::isfinite(p.beta) || p.beta < 0.0)
    return fail(MCLBM_EINVAL, "particle rho, cp, k must be > 0 and beta >= 0");
  if (c->force_mask > MCLBM_F_ALL) return fail(MCLBM_EINVAL, "unknown force bits");
  if (c->reading_flags & ~(unsigned)(MCLBM_R_LITERAL_K_RATIO | MCLBM_R_LITERAL_GRAVITY | MCLBM_R_COMMON_VELOCITY |
                                      MCLBM_R_GUO_FORCING | MCLBM_R_LITERAL_REACTIONS))
    return fail(MCLBM_EINVAL, "unknown reading flags");
  if (c->reading_flags & (MCLBM_R_GUO_FORCING | MCLBM_R_LITERAL_REACTIONS))
    return fail(MCLBM_EUNSUPPORTED, "reading flags GUO_FORCING and LITERAL_REACTIONS are not implemented");
  if (c->thermal_lattices < 0 || c->thermal_lattices > 2)
    return fail(MCLBM_EINVAL, "thermal_lattices must be 0, 1 or 2");
  if (c->thermal_lattices == 2 && c->storage != MCLBM_FP32S)
    return fail(MCLBM_EUNSUPPORTED, "two thermal lattices need FP32 storage");
  for (int k = 0; k < 6; ++k)
    if (!std::isfinite(c->force_scale[k])) return fail(MCLBM_EINVAL, "force_scale must be finite");
  if (!std::isfinite(c->phi_perturb_amp) || c->phi_perturb_amp < 0.0)
    return fail(MCLBM_EINVAL, "phi_perturb_amp must be >= 0");
  if (c->storage != MCLBM_FP32S && c->storage != MCLBM_FP16S && c->storage != MCLBM_BF16S)
    return fail(MCLBM_EINVAL, "unknown storage type");
  if (c->steps_per_launch < 0 || c->steps_per_launch > 2)
    return fail(MCLBM_EINVAL, "steps_per_launch must be 0, 1 or 2");
  if (c->steps_per_launch == 2 && !two_step_possible(*c))
    return fail(MCLBM_EUNSUPPORTED, "two steps per launch need one thermal lattice");
  const int bx = c->block_x == 0 ? 64 : c->block_x;
  const int by = c->block_y == 0 ? 1 : c->block_y;
  if (!(bx == 32 || bx == 64 || bx == 128 || bx == 256) || by < 1 ||
      !(bx * by == 64 || bx * by == 128 || bx * by == 256))
    return fail(MCLBM_EINVAL, "block shape must have block_x in {32,64,128,256} and 64..256 threads");
  return MCLBM_OK;
}

// Lattice units from Ra, Pr and tau_f: Eq 22 gives the lattice viscosity,
// Eq 16 (with base-fluid properties) the physical cavity width.
void derive(const mclbm_config& c, Derived& d) {
  double* v = d.v;
  const double nu_f = c.fluid.mu / c.fluid.rho;
  const double alpha_f = nu_f / c.Pr;
  const double N = (double)c.nx;
  double nu_L;
  if (c.tau_f > 0.0) {
    nu_L = (c.tau_f - 0.5) / 3.0;
  } else {
    // automatic: free-fall velocity sqrt(Ra nu alpha)/N at most 0.1 c_s
    const double cap = 0.1 / std::sqrt(3.0);
    const double s = std::sqrt(c.Ra / c.Pr) / N;  // free fall per unit nu
    nu_L = (0.1 * s > cap) ? cap / s : 0.1;
  }
  const double alpha_L = nu_L / c.Pr;
  const double H = c.Ra > 0.0
                       ? std::cbrt(c.Ra * nu_f * alpha_f / (kGravity * c.fluid.beta * c.dT_K))
                       : 0.01;
  const double dx = H / N;
  const double dt = nu_L * dx * dx / nu_f;
  const double R = c.particle.rho / c.fluid.rho;
  // Eq 10b at T0, Eq 10a constant with the ratio k_p/k_f (as printed,
  // k_f/k_p, with the literal reading flag)
  const double Re = c.fluid.rho * kBoltzmann * c.T0_K /
                    (3.0 * kPi * c.fluid.mu * c.fluid.mu * c.fluid.d_mol);
  const double kratio = (c.reading_flags & MCLBM_R_LITERAL_K_RATIO) ? c.fluid.k / c.particle.k
                                                                     : c.particle.k / c.fluid.k;
  const double Ck = 64.7 * std::pow(c.fluid.d_mol / c.dp_m, 0.369) * std::pow(kratio, 0.7476) *
                    std::pow(c.Pr, 0.995) * std::pow(Re, 1.2321);
  v[MCLBM_D_NU_L] = nu_L;
  v[MCLBM_D_ALPHA_L] = alpha_L;
  v[MCLBM_D_H] = H;
  v[MCLBM_D_DX] = dx;
  v[MCLBM_D_DT] = dt;
  v[MCLBM_D_G_L] = c.Ra * nu_L * alpha_L / (N * N * N);
  v[MCLBM_D_GRAV_L] = kGravity * dt * dt / dx;
  v[MCLBM_D_CK] = Ck;
  v[MCLBM_D_R] = R;
  v[MCLBM_D_TAU_F] = 3.0 * nu_L + 0.5;
  v[MCLBM_D_RHOC_RATIO] = (c.particle.rho * c.particle.cp) / (c.fluid.rho * c.fluid.cp);
  v[MCLBM_D_BETA_RATIO] = c.particle.beta / c.fluid.beta;
  v[MCLBM_D_RHO_F0] = 1.0 - c.phi0;
  v[MCLBM_D_RHO_P0] = R * c.phi0;
  v[MCLBM_D_NU_F] = nu_f;
  v[MCLBM_D_ALPHA_F] = alpha_f;
}

// Per-node coefficients of the fused step in lattice units (FP32 kernarg).
StepParams make_params(const mclbm_config& c, const Derived& D, const Layout& L) {
  const double* v = D.v;
  StepParams P{};
  P.nx = c.nx;
  P.ny = c.ny;
  P.px = L.px;
  P.plane = L.plane;
  // FP16 stores the deviations scaled by a power of two per lattice:
  // fluid and particle deviations (~1e-7 .. 2e-2) by 2^16, temperature
  // populations (|g| <= 0.25) by 2^12, keeping both ends inside the normal
  // range (6.1e-5 .. 65504).  FP32 and BF16 are unscaled.
  for (int l = 0; l < 3; ++l) {
    float sc = 1.0f;
    if (c.storage == MCLBM_FP16S) sc = l < 2 ? 65536.0f : 4096.0f;
    P.scale[l] = sc;
    P.inv_scale[l] = 1.0f / sc;
  }
  const double R = v[MCLBM_D_R], dx = v[MCLBM_D_DX], dt = v[MCLBM_D_DT], H = v[MCLBM_D_H];
  const double tau_f = v[MCLBM_D_TAU_F];
  const float rf_ref = (float)v[MCLBM_D_RHO_F0];
  const float rp_ref = (float)v[MCLBM_D_RHO_P0];
  P.rho_f_ref = rf_ref;
  P.rho_p_ref = rp_ref;
  // gravity reference: the fluid carries the weight of the uniform
  // suspension R phi0 (or nothing, with the literal reading of Table 1)
  const double gref = (c.reading_flags & MCLBM_R_LITERAL_GRAVITY) ? 0.0 : v[MCLBM_D_RHO_P0];
  P.dref_p = (float)((double)rp_ref - gref);
  P.rho_p0 = (float)gref;
  P.flags = (c.reading_flags & MCLBM_R_COMMON_VELOCITY) ? 1u : 0u;
  P.tau_f = (float)tau_f;
  P.omega_f = (float)(1.0 / tau_f);
  P.nl = lattices(c);
  // fluid thermal lattice (two thermal lattices): base-fluid diffusivity
  P.tau_thf = (float)(3.0 * v[MCLBM_D_ALPHA_L] + 0.5);
  P.omega_thf = (float)(1.0 / (3.0 * v[MCLBM_D_ALPHA_L] + 0.5));
  P.invR = (float)(1.0 / R);
  P.Rm1 = (float)(R - 1.0);
  P.crc = (float)(v[MCLBM_D_RHOC_RATIO] - 1.0);
  P.crb = (float)(v[MCLBM_D_BETA_RATIO] - 1.0);
  P.Ck = (float)v[MCLBM_D_CK];
  P.alpha3 = (float)(3.0 * v[MCLBM_D_ALPHA_L]);
  // Eq 23 solved for tau_p without cancellation:
  // tau_p - tau_f = (tau_f - 1/2) (r_mu - r_rho) / (r_rho rbar_p), with
  // (r_mu - r_rho)/rbar_p = (rho_m/R) (4.93 - (R - 1) + 222.4 phi).
  P.tp_a = (float)((tau_f - 0.5) / R);
  P.tp_b = (float)(4.93 - (R - 1.0));
  P.G_L = (float)v[MCLBM_D_G_L];

  double s[6];
  for (int k = 0; k < 6; ++k) s[k] = ((c.force_mask >> k) & 1u) ? c.force_scale[k] : 0.0;
  const double d = c.dp_m;
  const double Vp = kPi * d * d * d / 6.0, Ap = kPi * d * d, mp = c.particle.rho * Vp;
  const double mu = c.fluid.mu, rho = c.fluid.rho;
  const double dtdx2 = dt * dt / (dx * dx);
  // Brownian: rho_p D_B A_p v_B / m_p = 8 kB^2 T^2 / (pi^2 mu^2 d^4) per grad phi
  P.cB = (float)(s[1] * 8.0 * kBoltzmann * kBoltzmann * c.T0_K * c.T0_K /
                 (kPi * kPi * mu * mu * d * d * d * d) * dtdx2);
  // thermophoresis: mu_ns d v_T / m_p with v_T = C_T (mu/rho)_ns grad T / T
  P.cT = (float)(s[2] * mu * mu * d * c.dT_K / (mp * rho * c.T0_K) * dtdx2);
  const double Kn = c.fluid.d_mol / d;
  P.kfp = (float)(c.fluid.k / c.particle.k);
  P.A1 = (float)(kCt * Kn);
  P.A2 = (float)(6.0 * kPi * kCs / (1.0 + 3.0 * kCm * Kn));
  P.dT_T0 = (float)(c.dT_K / c.T0_K);
  // Saffman: (K_S/4) mu |w| d^2 sqrt(rho gdot / mu) / m_p, gdot = 8 |v_p| / H
  P.cS = (float)(s[3] * (kKs / 4.0) * d * d * dt * std::sqrt(8.0 * mu * rho * dx / (dt * H)) / mp);
  // Magnus: (|v_M|/d)(v_p - v_M); rotation: mu rho_p gdot A_p / (rho m_p)
  P.cM = (float)(s[4] * dx / d);
  P.cR = (float)(s[4] * 8.0 * R * mu * Ap * dt / (H * mp));
  // settling -(1 - rho_f/rho_p) g (the fluid carries R phi0 (1 - 1/R) g)
  P.cG = (float)(s[5] * (1.0 - 1.0 / R) * v[MCLBM_D_GRAV_L]);
  // drag: Re_d = rho_p d |w| / mu_ns, beta = 18 mu_ns (1 + 0.15 Re^0.687)/(rho_p d^2)
  P.cRe = (float)(c.particle.rho * d * (dx / dt) / mu);
  P.cD = (float)(s[0] * 18.0 * mu * dt / (c.particle.rho * d * d));
  unsigned on = 0;
  if (P.cD != 0.0f) on |= 1u;
  if (P.cB != 0.0f) on |= 2u;
  if (P.cT != 0.0f) on |= 4u;
  if (P.cS != 0.0f) on |= 8u;
  if (P.cM != 0.0f || P.cR != 0.0f) on |= 16u;
  if (P.cG != 0.0f) on |= 32u;
  P.force_on = on;
  return P;
}

}  // namespace

// ---- static scratch of the allocation-free residual -------------------------
// mclbm_residual_noalloc keeps its per-block FP64 partials here instead of in
// the cavity's buffer: one copy of the array per GPU, held for the life of
// the process.  In host code `scratch` names a host-side stand-in, not a
// device address; host code uses only the address resolved per device by
// noalloc_scratch().
static __device__ __align__(256) double scratch[MCLBM_NOALLOC_SCRATCH_BYTES / sizeof(double)];

struct mclbm_cavity {
  mclbm_config cfg;
  std::vector<double> xi;
  hipStream_t stream;
  char* base;
  size_t bytes;
  Layout L;
  Derived D;
  StepParams P;
  int64_t t;
  dim3 block;          // step-kernel workgroup shape
  unsigned nblocks;    // step-kernel 1-D grid (tiles)
  int tiles_x;
  bool nt;             // non-temporal population traffic
  bool idx32;          // 32-bit element offsets
  bool in_batch;       // owned by a batch: stepped only through it
  bool pad_planes;     // planes padded at any size (members of a streaming batch)
  bool poison;         // race check: NaN-fill what a step writes before it runs
  bool two;            // two steps per launch (k_step2) from even steps
  int popsel, d2sel;   // which population copy is current; lag-field swap
  unsigned nblocks2;   // k_step2 grid: strips x bands
  int mix2;            // k_step2 band interleave (band_of_tile)
  int strips2, band2;
  const int64_t* batch_clock;  // the owning batch's step count (members only)
  std::vector<double> host_dev_p;  // initial phi deviations (source of an async copy)
  int device = -1;     // HIP device current at creation
  uint64_t epoch = 0;  // bumped by every change of state other than stepping
  int32_t nu_every = 0;   // record the Nusselt numbers every nu_every steps (0: off)
  double* nu_ring = nullptr;
  int32_t nu_cap = 0;
  int64_t nu_count = 0;   // records written since recording was enabled

  size_t pop_off(int k) const { return k ? L.off_pop2 : L.off_pop; }
  void* pop() { return base + pop_off(popsel); }
  void* pop_other() { return base + pop_off(popsel ^ 1); }
  size_t d2_off(int k) const { return L.off_d2 + (size_t)(k ^ d2sel) * L.plane * sizeof(float2); }
  float2* d2(int k) { return reinterpret_cast<float2*>(base + d2_off(k)); }
  float* d5() { return reinterpret_cast<float*>(base + L.off_d5); }
  double* snap() { return reinterpret_cast<double*>(base + L.off_snap); }
  double* part() { return reinterpret_cast<double*>(base + L.off_part); }
  double* res() { return reinterpret_cast<double*>(base + L.off_res); }
  double* stage() { return reinterpret_cast<double*>(base + L.off_stage); }
};

namespace {

int launch_check(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, what);
  return MCLBM_OK;
}

// Kernel type selection: storage format S (cached access, auxiliary
// kernels), the access policies of the even (SE) and odd (SO) step kernels,
// and the index type I.  Above the last-level cache the even step streams
// loads and stores past the caches; the odd step streams its loads but
// keeps its stores cached: they are shifted by one node, so the edge lines
// of two neighbouring workgroups are each written half by either, and L2
// merges the halves instead of sending two partial lines to HBM.
template <class S_, class SE_, class SO_, class I_, int NL_ = 3>
struct KTypes {
  using S = S_;
  using SE = SE_;
  using SO = SO_;
  using I = I_;
  static constexpr int NL = NL_;  // lattices: 3, or 4 with two thermal lattices
};

template <template <bool, bool> class St, int NL = 3, class Fn>
int dispatch_storage(bool idx32, bool nt, Fn&& fn) {
  using C = St<false, false>;
  using E = St<true, true>;
  using O = St<true, false>;
  if (idx32) {
    if (nt) return fn(KTypes<C, E, O, uint32_t, NL>{});
    return fn(KTypes<C, C, C, uint32_t, NL>{});
  }
  if (nt) return fn(KTypes<C, E, O, uint64_t, NL>{});
  return fn(KTypes<C, C, C, uint64_t, NL>{});
}

template <bool L, bool S>
using F32 = StorF32<L, S>;
template <bool L, bool S>
using F16 = StorF16<L, S>;
template <bool L, bool S>
using BF16 = StorBF16<L, S>;

template <class Fn>
int dispatch_kinds(int storage, bool idx32, bool nt, Fn&& fn) {
  switch (storage) {
    case MCLBM_FP32S: return dispatch_storage<F32>(idx32, nt, fn);
    case MCLBM_FP16S: return dispatch_storage<F16>(idx32, nt, fn);
    case MCLBM_BF16S: return dispatch_storage<BF16>(idx32, nt, fn);
    default: return fail(MCLBM_EUNSUPPORTED, "unknown storage type");
  }
}

template <class Fn>
int dispatch(const mclbm_cavity* c, Fn&& fn) {
  if (c->P.nl == 4) {
    // two thermal lattices: FP32 storage only (checked at creation)
    if (c->cfg.storage != MCLBM_FP32S) return fail(MCLBM_EUNSUPPORTED, "four lattices need FP32 storage");
    return dispatch_storage<F32, 4>(c->idx32, c->nt, fn);
  }
  return dispatch_kinds(c->cfg.storage, c->idx32, c->nt, fn);
}

// Grid over all nodes for the auxiliary kernels.
unsigned node_blocks(const mclbm_cavity* c) {
  return (unsigned)(((long long)c->cfg.nx * c->cfg.ny + 255) / 256);
}

int enqueue_init(mclbm_cavity* c) {
  ++c->epoch;
  const mclbm_config& cfg = c->cfg;
  const long long nn = (long long)cfg.nx * cfg.ny;
  const double R = c->D.v[MCLBM_D_R];
  const double rp_ref = (double)c->P.rho_p_ref;
  c->host_dev_p.assign((size_t)nn, 0.0);
  for (long long k = 0; k < nn; ++k) {
    double phi = cfg.phi0;
    if (!c->xi.empty()) phi += cfg.phi_perturb_amp * c->xi[(size_t)k];
    if (phi < 0.0) phi = 0.0;
    c->host_dev_p[(size_t)k] = R * phi - rp_ref;
  }
  const double dev_f = c->D.v[MCLBM_D_RHO_F0] - (double)c->P.rho_f_ref;
  HIP_TRY(hipMemcpyAsync(c->stage(), c->host_dev_p.data(), (size_t)nn * sizeof(double),
                         hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipMemsetAsync(c->d5(), 0, (size_t)6 * (c->P.nl - 2) * c->L.px * sizeof(float), c->stream));
  int rc = dispatch(c, [&](auto k) {
    using S = typename decltype(k)::S;
    using I = typename decltype(k)::I;
    auto* pop = reinterpret_cast<typename S::T*>(c->pop());
    const dim3 b2(64, 4, 1), g2((cfg.nx + 63) / 64, (cfg.ny + 3) / 4, 1);
    k_init<S, decltype(k)::NL><<<g2, b2, 0, c->stream>>>(c->P, pop, c->stage(), dev_f, c->d2(1));
    int r = launch_check("k_init");
    if (r) return r;
    // snapshot of the initial state for the first residual call
    k_residual<false, S, I, decltype(k)::NL><<<c->L.red_blocks, 256, 0, c->stream>>>(
        c->P, pop, c->d5(), (double)c->P.rho_f_ref, (double)c->P.rho_p_ref, c->snap(), c->part());
    return launch_check("k_residual");
  });
  if (rc) return rc;
  c->t = 0;
  HIP_TRY(hipStreamSynchronize(c->stream));
  return MCLBM_OK;
}

bool env_flag(const char* name) {
  const char* v = std::getenv(name);
  return v && v[0] == '1';
}

int setup_cavity(mclbm_cavity* c) {
  derive(c->cfg, c->D);
  c->L = make_layout(c->cfg, c->in_batch, c->pad_planes);
  c->P = make_params(c->cfg, c->D, c->L);
  int bx = c->cfg.block_x, by = c->cfg.block_y;
  // Default workgroup: 256 x 1 from 256 columns on; with 16-bit storage
  // 64 x 1 from 2^21 nodes on (2048^2 and 4096^2: +3-4 % over 256 x 1 for
  // FP16 and BF16; equal at 1024^2, 3.5 % slower at 512^2; FP32 is fastest
  // with 256 x 1 at every size).
  const bool narrow16 = c->cfg.storage != MCLBM_FP32S && (long long)c->cfg.nx * c->cfg.ny >= (1LL << 21);
  if (bx == 0) bx = c->cfg.nx >= 256 && !narrow16 ? 256 : 64;
  if (by == 0) by = 1;
  c->block = dim3(bx, by, 1);
  c->tiles_x = (c->cfg.nx + bx - 1) / bx;
  c->nblocks = (unsigned)c->tiles_x * (unsigned)((c->cfg.ny + by - 1) / by);
  const size_t pop_bytes = (size_t)9 * c->P.nl * c->L.plane * storage_bytes(c->cfg.storage);
  c->nt = pop_bytes + (size_t)2 * c->L.plane * sizeof(float2) > kStreamingBytes;
  c->idx32 = pop_bytes < ((size_t)1 << 31);
  // Test knobs: the 64-bit index path and the streaming access policy are
  // otherwise taken only by cavities above 2 GiB or 160 MiB; the results do
  // not depend on either, which the tests check on small cavities.
  if (env_flag("MCLBM_INDEX64")) c->idx32 = false;
  if (env_flag("MCLBM_STREAMING")) c->nt = true;
  c->poison = env_flag("MCLBM_POISON");
  // two steps per launch: strips of kStrip2 columns, bands of band2 rows
  c->two = two_step(c->cfg, c->in_batch) && (c->idx32 || !c->in_batch);
  c->strips2 = strips2_of(c->cfg);
  c->band2 = band2_of(c->cfg);
  c->mix2 = mix2_of(c->cfg);
  c->nblocks2 = (unsigned)c->strips2 * (unsigned)((c->cfg.ny + c->band2 - 1) / c->band2);
  return MCLBM_OK;
}

template <class K>
int launch_step(mclbm_cavity* c) {
  using I = typename K::I;
  using T = typename K::S::T;
  auto* pop = reinterpret_cast<T*>(c->pop());
  if (c->poison) {
    // race check: what this step writes and must not read first is NaN
    // (the lag field it stores; before an even step the side buffer the
    // odd step reads), so a read before the write shows up in the results
    const long long n2 = 2 * c->L.plane;
    k_poison<<<(unsigned)std::min<long long>((n2 + 255) / 256, 65536), 256, 0, c->stream>>>(
        reinterpret_cast<float*>(c->d2((c->t & 1) ? 1 : 0)), n2);
    if ((c->t & 1) == 0) {
      const long long n5 = 6LL * (c->P.nl - 2) * c->L.px;
      k_poison<<<(unsigned)((n5 + 255) / 256), 256, 0, c->stream>>>(c->d5(), n5);
    }
    int r = launch_check("k_poison");
    if (r) return r;
  }
  if ((c->t & 1) == 0)
    k_step<false, typename K::SE, I, K::NL><<<c->nblocks, c->block, 0, c->stream>>>(c->P, pop, c->d2(1), c->d2(0),
                                                                           c->d5(), c->tiles_x);
  else
    k_step<true, typename K::SO, I, K::NL><<<c->nblocks, c->block, 0, c->stream>>>(c->P, pop, c->d2(0), c->d2(1),
                                                                          c->d5(), c->tiles_x);
  return launch_check("k_step");
}

// Steps t (even) and t + 1 in one launch, from the current population copy
// into the other one; the lag field of t + 1 goes to the buffer that held the
// one of t - 1's partner, and both selections flip.
template <class K>
int launch_step2(mclbm_cavity* c) {
  if constexpr (K::NL == 3) {
    // cached loads and stores at every size: a wave's 64 lanes start one
    // column before its strip, so its row loads straddle the cache lines it
    // shares with the neighbouring strips (and bands), which then hit in L2;
    // non-temporal loads evict them first and read 1.64x the bytes
    using S = typename K::S;
    using T = typename S::T;
    auto* src = reinterpret_cast<const T*>(c->pop());
    auto* dst = reinterpret_cast<T*>(c->pop_other());
    if (c->poison) {
      // race check: every slot of the target copy and every lag-field entry
      // the launch writes start as NaN, so a slot left unwritten (or read
      // before it is written) shows up in the results
      const long long np = (long long)pop_bytes(c->cfg, c->L.plane) / (long long)sizeof(float);
      k_poison<<<(unsigned)std::min<long long>((np + 255) / 256, 1 << 20), 256, 0, c->stream>>>(
          reinterpret_cast<float*>(c->pop_other()), np);
      const long long n2 = 2 * c->L.plane;
      k_poison<<<(unsigned)std::min<long long>((n2 + 255) / 256, 65536), 256, 0, c->stream>>>(
          reinterpret_cast<float*>(c->d2(0)), n2);
      int r = launch_check("k_poison");
      if (r) return r;
    }
    k_step2<S, typename K::I><<<c->nblocks2, 64, 0, c->stream>>>(c->P, src, dst, c->d2(1), c->d2(0), c->strips2,
                                                                 c->band2, c->mix2);
    int r = launch_check("k_step2");
    if (r) return r;
    c->popsel ^= 1;
    c->d2sel ^= 1;
    return MCLBM_OK;
  } else {
    return fail(MCLBM_EUNSUPPORTED, "two steps per launch: one thermal lattice only");
  }
}

int export_pops(mclbm_cavity* c, int q, double* dev_out) {
  const double rf = (double)c->P.rho_f_ref, rp = (double)c->P.rho_p_ref;
  return dispatch(c, [&](auto k) {
    using S = typename decltype(k)::S;
    using I = typename decltype(k)::I;
    const auto* pop = reinterpret_cast<const typename S::T*>(c->pop());
    if (c->t & 1)
      k_export_pops<true, S, I, decltype(k)::NL><<<node_blocks(c), 256, 0, c->stream>>>(c->P, pop, c->d5(), rf, rp, q, dev_out);
    else
      k_export_pops<false, S, I, decltype(k)::NL><<<node_blocks(c), 256, 0, c->stream>>>(c->P, pop, c->d5(), rf, rp, q, dev_out);
    return launch_check("k_export_pops");
  });
}

int enqueue_load_fields(mclbm_cavity* c, const float* F, int sx, int sy, int nc, const double* affine) {
  ++c->epoch;
  const mclbm_config& cfg = c->cfg;
  const long long nn = (long long)cfg.nx * cfg.ny;
  FieldMap M{};
  M.F = F;
  M.sx = sx;
  M.sy = sy;
  M.nc = nc;
  for (int q = 0; q < nc; ++q) {
    M.a[q] = affine ? affine[q] : 1.0;
    M.b[q] = affine ? affine[nc + q] : 0.0;
  }
  // particle inventory of the cold start (the initial state of mclbm_create)
  double inventory = 0.0;
  for (long long k = 0; k < nn; ++k) {
    double phi = cfg.phi0;
    if (!c->xi.empty()) phi += cfg.phi_perturb_amp * c->xi[(size_t)k];
    inventory += phi < 0.0 ? 0.0 : phi;
  }
  LoadConst K{};
  K.inventory = inventory;
  K.rho_f0 = c->D.v[MCLBM_D_RHO_F0];
  K.R = c->D.v[MCLBM_D_R];
  K.tau_f = c->D.v[MCLBM_D_TAU_F];
  K.alpha3 = 3.0 * c->D.v[MCLBM_D_ALPHA_L];
  K.Ck = c->D.v[MCLBM_D_CK];
  K.crc_m1 = c->D.v[MCLBM_D_RHOC_RATIO] - 1.0;
  HIP_TRY(hipMemsetAsync(c->d5(), 0, (size_t)6 * (c->P.nl - 2) * c->L.px * sizeof(float), c->stream));
  k_load_sums<<<c->L.red_blocks, 256, 0, c->stream>>>(M, cfg.nx, cfg.ny, c->part());
  int rc = launch_check("k_load_sums");
  if (rc) return rc;
  k_sum_partials<<<1, 256, 0, c->stream>>>(c->part(), c->L.red_blocks, c->res());
  rc = launch_check("k_sum_partials");
  if (rc) return rc;
  rc = dispatch(c, [&](auto k) {
    using S = typename decltype(k)::S;
    using I = typename decltype(k)::I;
    auto* pop = reinterpret_cast<typename S::T*>(c->pop());
    k_load_fields<S><<<node_blocks(c), 256, 0, c->stream>>>(c->P, M, K, pop, c->res(), c->d2(1));
    int r = launch_check("k_load_fields");
    if (r) return r;
    k_residual<false, S, I, decltype(k)::NL><<<c->L.red_blocks, 256, 0, c->stream>>>(
        c->P, pop, c->d5(), (double)c->P.rho_f_ref, (double)c->P.rho_p_ref, c->snap(), c->part());
    return launch_check("k_residual");
  });
  if (rc) return rc;
  c->t = 0;
  HIP_TRY(hipStreamSynchronize(c->stream));
  return MCLBM_OK;
}

// The FP64 reductions in two halves: enqueue the kernels and the copy of
// their results to host memory `h` (pinned for an asynchronous copy), then,
// after the stream has been synchronised, read them.  A batch enqueues all
// its cavities before one synchronisation.
// The Nusselt numbers of the current state into device memory `out` (4
// doubles: hot, cold, hot conductivity-weighted, non-finite flag).  Async.
int launch_nusselt(mclbm_cavity* c, double* out) {
  const double rp = (double)c->P.rho_p_ref, R = c->D.v[MCLBM_D_R], Ck = c->D.v[MCLBM_D_CK];
  return dispatch(c, [&](auto k) {
    using S = typename decltype(k)::S;
    using I = typename decltype(k)::I;
    const auto* pop = reinterpret_cast<const typename S::T*>(c->pop());
    if (c->t & 1)
      k_nusselt<true, S, I, decltype(k)::NL><<<1, 256, 0, c->stream>>>(c->P, pop, c->d5(), rp, R, Ck, out);
    else
      k_nusselt<false, S, I, decltype(k)::NL><<<1, 256, 0, c->stream>>>(c->P, pop, c->d5(), rp, R, Ck, out);
    return launch_check("k_nusselt");
  });
}

int enqueue_nusselt(mclbm_cavity* c, double* h) {
  int rc = launch_nusselt(c, c->res());
  if (rc) return rc;
  HIP_TRY(hipMemcpyAsync(h, c->res(), 4 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  return MCLBM_OK;
}

int finish_nusselt(const double* h, double* nu_hot, double* nu_cold, double* nu_hot_k) {
  if (nu_hot) *nu_hot = h[0];
  if (nu_cold) *nu_cold = h[1];
  if (nu_hot_k) *nu_hot_k = h[2];
  if (h[3] != 0.0) return fail(MCLBM_EDIVERGED, "non-finite temperature at a wall");
  return MCLBM_OK;
}

// Per-block partial sums of the residual into `part` (5 doubles per block
// of 256 nodes); the snapshot becomes the current state.
int enqueue_residual_partials(mclbm_cavity* c, double* part) {
  const unsigned rb = (unsigned)c->L.red_blocks;
  const double rf = (double)c->P.rho_f_ref, rp = (double)c->P.rho_p_ref;
  return dispatch(c, [&](auto k) {
    using S = typename decltype(k)::S;
    using I = typename decltype(k)::I;
    const auto* pop = reinterpret_cast<const typename S::T*>(c->pop());
    if (c->t & 1)
      k_residual<true, S, I, decltype(k)::NL><<<rb, 256, 0, c->stream>>>(c->P, pop, c->d5(), rf, rp, c->snap(), part);
    else
      k_residual<false, S, I, decltype(k)::NL><<<rb, 256, 0, c->stream>>>(c->P, pop, c->d5(), rf, rp, c->snap(), part);
    return launch_check("k_residual");
  });
}

int enqueue_residual(mclbm_cavity* c, double* h) {
  const unsigned rb = (unsigned)c->L.red_blocks;
  int rc = enqueue_residual_partials(c, c->part());
  if (rc) return rc;
  k_sum_partials<<<1, 256, 0, c->stream>>>(c->part(), (int)rb, c->res() + 4);
  rc = launch_check("k_sum_partials");
  if (rc) return rc;
  HIP_TRY(hipMemcpyAsync(h, c->res() + 4, 5 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  return MCLBM_OK;
}

// Device address of `scratch` on device `dev` (which must be current),
// resolved once per device and kept.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

int noalloc_scratch(int dev, double** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(MCLBM_EINVAL, "device ordinal out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return MCLBM_OK;
}

// Set-up step of a cavity: record its device and resolve that device's
// scratch address while no stream capture can be running.  A failure here
// is reported by the first mclbm_residual_noalloc call instead.
void setup_device(mclbm_cavity* c) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return;
  c->device = dev;
  double* unused = nullptr;
  (void)noalloc_scratch(dev, &unused);
  (void)hipGetLastError();
}

int finish_residual(const double* h, double* res_u, double* res_theta) {
  const double ru = h[1] > 0.0 ? std::sqrt(h[0] / h[1]) : (h[0] > 0.0 ? INFINITY : 0.0);
  const double rt = h[3] > 0.0 ? std::sqrt(h[2] / h[3]) : (h[2] > 0.0 ? INFINITY : 0.0);
  if (res_u) *res_u = ru;
  if (res_theta) *res_theta = rt;
  if (h[4] != 0.0) return fail(MCLBM_EDIVERGED, "non-finite velocity or temperature");
  return MCLBM_OK;
}

}  // namespace

// ---- checkpoint / resume ----------------------------------------------------
namespace {

constexpr int kCkptVersion = 2;

// A section of the file: `bytes` in `rows` equal rows, which lie `pitch`
// bytes apart in device memory.  The file holds the planes without the pad
// between them (px * ny elements each), so a checkpoint does not depend on
// the plane pad of the cavity that wrote it.
struct CkptSection {
  const char* name;
  size_t off, bytes;
  size_t rows, pitch;
};

std::vector<CkptSection> ckpt_sections(const mclbm_cavity* c) {
  const long long nn = (long long)c->cfg.nx * c->cfg.ny;
  const size_t lp = (size_t)c->L.px * c->cfg.ny;  // elements of a plane without its pad
  const size_t sb = storage_bytes(c->cfg.storage);
  const size_t np = (size_t)9 * c->P.nl;
  return {
      {"populations", c->pop_off(c->popsel), np * lp * sb, np, (size_t)c->L.plane * sb},
      {"lag_field_0", c->d2_off(0), lp * sizeof(float2), 1, 0},
      {"lag_field_1", c->d2_off(1), lp * sizeof(float2), 1, 0},
      {"side_buffer", c->L.off_d5, (size_t)6 * (c->P.nl - 2) * c->L.px * sizeof(float), 1, 0},
      {"residual_snapshot", c->L.off_snap, (size_t)3 * nn * sizeof(double), 1, 0},
  };
}

// Copies of one section between the device and the host (sync).
hipError_t ckpt_to_host(const mclbm_cavity* c, const CkptSection& sc, void* host) {
  if (sc.rows <= 1) return hipMemcpy(host, c->base + sc.off, sc.bytes, hipMemcpyDeviceToHost);
  const size_t w = sc.bytes / sc.rows;
  return hipMemcpy2D(host, w, c->base + sc.off, sc.pitch, w, sc.rows, hipMemcpyDeviceToHost);
}
hipError_t ckpt_to_device(mclbm_cavity* c, const CkptSection& sc, const void* host) {
  if (sc.rows <= 1) return hipMemcpy(c->base + sc.off, host, sc.bytes, hipMemcpyHostToDevice);
  const size_t w = sc.bytes / sc.rows;
  return hipMemcpy2D(c->base + sc.off, sc.pitch, host, w, w, sc.rows, hipMemcpyHostToDevice);
}

std::string hex_of(const void* p, size_t n) {
  static const char* d = "0123456789abcdef";
  std::string s;
  s.reserve(2 * n);
  const unsigned char* b = static_cast<const unsigned char*>(p);
  for (size_t k = 0; k < n; ++k) {
    s.push_back(d[b[k] >> 4]);
    s.push_back(d[b[k] & 15]);
  }
  return s;
}

// The configuration a checkpoint is tied to: the physics, not the launch
// shape (workgroup shape, steps per launch), which leaves the state alone.
std::string config_key(const mclbm_config& c) {
  mclbm_config k = c;
  k.block_x = k.block_y = 0;
  k.steps_per_launch = 0;
  return hex_of(&k, sizeof k);
}

std::string json_string_field(const std::string& h, const char* key) {
  const std::string k = std::string("\"") + key + "\": \"";
  const size_t a = h.find(k);
  if (a == std::string::npos) return "";
  const size_t b = h.find('"', a + k.size());
  return b == std::string::npos ? "" : h.substr(a + k.size(), b - a - k.size());
}

bool json_number_field(const std::string& h, const char* key, long long& v) {
  const std::string k = std::string("\"") + key + "\": ";
  const size_t a = h.find(k);
  if (a == std::string::npos) return false;
  char* end = nullptr;
  v = std::strtoll(h.c_str() + a + k.size(), &end, 10);
  return end != h.c_str() + a + k.size();
}

// Decode a lowercase hex string into exactly n bytes (false on any other
// length or character).
bool unhex(const std::string& s, void* out, size_t n) {
  if (s.size() != 2 * n) return false;
  unsigned char* b = static_cast<unsigned char*>(out);
  for (size_t k = 0; k < n; ++k) {
    int v = 0;
    for (int q = 0; q < 2; ++q) {
      const char ch = s[2 * k + q];
      const int d = (ch >= '0' && ch <= '9') ? ch - '0' : ((ch >= 'a' && ch <= 'f') ? ch - 'a' + 10 : -1);
      if (d < 0) return false;
      v = 16 * v + d;
    }
    b[k] = (unsigned char)v;
  }
  return true;
}

// The header line of a checkpoint file and what it names: the physics
// configuration (launch shape zeroed), the initial perturbation field (empty
// if the cavity had none) and the step count.  Leaves fp after the header.
struct CkptHeader {
  std::string line;
  mclbm_config cfg;
  std::vector<double> xi;
  long long t = -1;
};

int read_ckpt_header(FILE* fp, CkptHeader& H) {
  H.line.clear();
  for (int ch; (ch = std::fgetc(fp)) != EOF && ch != '\n';) {
    H.line.push_back((char)ch);
    if (H.line.size() > (64u << 20)) return fail(MCLBM_EINVAL, "checkpoint: header line too long");
  }
  long long ver = 0;
  if (json_string_field(H.line, "format") != "mclbm-checkpoint" || !json_number_field(H.line, "version", ver) ||
      ver != kCkptVersion)
    return fail(MCLBM_EINVAL, "checkpoint: not a checkpoint of this format");
  if (!unhex(json_string_field(H.line, "config_hex"), &H.cfg, sizeof H.cfg))
    return fail(MCLBM_EINVAL, "checkpoint: damaged configuration");
  if (validate(&H.cfg) != MCLBM_OK) return fail(MCLBM_EINVAL, "checkpoint: invalid configuration");
  const std::string xh = json_string_field(H.line, "xi_hex");
  const size_t nn = (size_t)H.cfg.nx * (size_t)H.cfg.ny;
  H.xi.clear();
  if (!xh.empty()) {
    H.xi.resize(nn);
    if (!unhex(xh, H.xi.data(), nn * sizeof(double)))
      return fail(MCLBM_EINVAL, "checkpoint: damaged initial perturbation field");
  }
  if (!json_number_field(H.line, "t", H.t) || H.t < 0) return fail(MCLBM_EINVAL, "checkpoint: no step count");
  return MCLBM_OK;
}

// MCLBM_LOG=debug: one line per configuration on stderr with the lattice
// constants and the stability numbers at the initial state (phi = phi0,
// theta = 0, at rest): tau_p and tau_theta (Eqs 23-24), g beta dT (Eq 16),
// dx, dt, the Mach number of the free-fall velocity sqrt(g beta dT N) and
// the drag stiffness kappa = beta dt (1 + rho_p / rho_f).
void log_derived(const mclbm_config& c, const Derived& D) {
  const char* e = std::getenv("MCLBM_LOG");
  if (!e || std::strcmp(e, "debug") != 0) return;
  const StepParams P = make_params(c, D, make_layout(c));
  const double phi = c.phi0, R = D.v[MCLBM_D_R];
  const double r_rho = 1.0 + phi * (R - 1.0), r_rhoc = 1.0 + phi * P.crc;
  const double r_mu = 1.0 + 4.93 * phi + 222.4 * phi * phi;
  const double r_k = 1.0 + D.v[MCLBM_D_CK] * std::pow(phi, 0.764);
  const double rho_f = D.v[MCLBM_D_RHO_F0], rho_p = D.v[MCLBM_D_RHO_P0], rho_m = rho_f + rho_p;
  double tau_p = P.tau_f + P.tp_a * rho_m * (P.tp_b + 222.4 * phi) / r_rho;
  tau_p = std::min(std::max(tau_p, 0.505), 5.0);
  const double tau_th = 3.0 * D.v[MCLBM_D_ALPHA_L] * r_k / r_rhoc + 0.5;
  const double u_ff = std::sqrt(std::max(D.v[MCLBM_D_G_L], 0.0) * c.nx);
  const double kappa = (double)P.cD * r_mu * (1.0 + (rho_f > 0.0 ? rho_p / rho_f : 0.0));
  std::fprintf(stderr,
               "mclbm: nx %d ny %d Ra %.6g phi0 %.6g dp_m %.6g | tau_f %.6g tau_p %.6g tau_theta %.6g "
               "G_L %.6g dx %.6g dt %.6g | Mach %.4g kappa %.6g\n",
               c.nx, c.ny, c.Ra, c.phi0, c.dp_m, (double)P.tau_f, tau_p, tau_th, D.v[MCLBM_D_G_L],
               D.v[MCLBM_D_DX], D.v[MCLBM_D_DT], u_ff * std::sqrt(3.0), kappa);
  std::fflush(stderr);
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================

namespace {
template <class SS>
int launch_convert(mclbm_cavity* dst, const mclbm_cavity* src, long long n) {
  const auto* from = reinterpret_cast<const typename SS::T*>(const_cast<mclbm_cavity*>(src)->pop());
  const unsigned grid = (unsigned)std::min<long long>((n + 255) / 256, 1 << 16);
  switch (dst->cfg.storage) {
    case MCLBM_FP32S:
      k_convert<SS, StorF32<false>><<<grid, 256, 0, dst->stream>>>(
          from, reinterpret_cast<float*>(dst->pop()), dst->L.plane, n, src->P, dst->P);
      break;
    case MCLBM_FP16S:
      k_convert<SS, StorF16<false>><<<grid, 256, 0, dst->stream>>>(
          from, reinterpret_cast<__half*>(dst->pop()), dst->L.plane, n, src->P, dst->P);
      break;
    default:
      k_convert<SS, StorBF16<false>><<<grid, 256, 0, dst->stream>>>(
          from, reinterpret_cast<__hip_bfloat16*>(dst->pop()), dst->L.plane, n, src->P, dst->P);
  }
  return launch_check("k_convert");
}
}  // namespace

extern "C" {

void mclbm_config_defaults(mclbm_config* c) {
  if (!c) return;
  std::memset(c, 0, sizeof(*c));
  c->nx = c->ny = 64;
  c->Ra = 1e3;
  c->Pr = 6.2;
  c->phi0 = 0.01;
  c->dp_m = 100e-9;
  c->tau_f = 0.8;
  c->dT_K = 10.0;
  c->T0_K = 300.0;
  c->force_mask = MCLBM_F_ALL;
  for (int k = 0; k < 6; ++k) c->force_scale[k] = 1.0;
  c->phi_perturb_amp = 1e-6;
  // water and alumina near 300 K
  c->fluid = mclbm_material{997.1, 4179.0, 0.613, 2.1e-4, 8.9e-4, 0.384e-9};
  c->particle = mclbm_material{3970.0, 765.0, 40.0, 8.5e-6, 0.0, 0.0};
  c->storage = MCLBM_FP32S;
  c->block_x = 0;
  c->block_y = 0;
  c->thermal_lattices = 1;
}

size_t mclbm_device_bytes(const mclbm_config* cfg) {
  if (validate(cfg) != MCLBM_OK) return 0;
  return make_layout(*cfg).total;
}

int mclbm_derive_constants(const mclbm_config* cfg, double* out, int n) {
  int rc = validate(cfg);
  if (rc) return rc;
  if (!out || n < MCLBM_D_COUNT) return fail(MCLBM_EINVAL, "output too small");
  Derived d;
  derive(*cfg, d);
  std::memcpy(out, d.v, sizeof(d.v));
  log_derived(*cfg, d);
  return MCLBM_OK;
}

int mclbm_create(const mclbm_config* cfg, const double* xi_host, void* dev_buf, size_t bytes,
                 void* stream, mclbm_cavity** out) {
  if (!out) return fail(MCLBM_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = validate(cfg);
  if (rc) return rc;
  if (!dev_buf) return fail(MCLBM_EINVAL, "dev_buf is NULL");
  if (reinterpret_cast<uintptr_t>(dev_buf) % kAlign != 0)
    return fail(MCLBM_EINVAL, "dev_buf must be 256-byte aligned");
  const size_t need = make_layout(*cfg).total;
  if (bytes < need)
    return fail(MCLBM_ENOMEM, "device buffer too small: need " + std::to_string(need) + " bytes");
  mclbm_cavity* c = new (std::nothrow) mclbm_cavity();
  if (!c) return fail(MCLBM_ENOMEM, "host allocation failed");
  c->cfg = *cfg;
  if (xi_host) c->xi.assign(xi_host, xi_host + (size_t)cfg->nx * cfg->ny);
  c->stream = reinterpret_cast<hipStream_t>(stream);
  c->base = reinterpret_cast<char*>(dev_buf);
  c->bytes = bytes;
  setup_cavity(c);
  setup_device(c);
  log_derived(c->cfg, c->D);
  rc = enqueue_init(c);
  if (rc) {
    delete c;
    return rc;
  }
  *out = c;
  return MCLBM_OK;
}

int mclbm_set_properties(mclbm_cavity* c, double Ra, double phi0, double dp_m) {
  if (!c) return fail(MCLBM_EINVAL, "cavity is NULL");
  if (c->in_batch) return fail(MCLBM_ESTATE, "cavity belongs to a batch: use the batch calls");
  mclbm_config nc = c->cfg;
  nc.Ra = Ra;
  nc.phi0 = phi0;
  nc.dp_m = dp_m;
  int rc = validate(&nc);
  if (rc) return rc;
  c->cfg = nc;
  setup_cavity(c);
  return enqueue_init(c);
}

int mclbm_reset(mclbm_cavity* c) {
  if (!c) return fail(MCLBM_EINVAL, "cavity is NULL");
  if (c->in_batch) return fail(MCLBM_ESTATE, "cavity belongs to a batch: use the batch calls");
  return enqueue_init(c);
}

int mclbm_load_fields(mclbm_cavity* c, const float* dev_fields, int32_t sx, int32_t sy, int32_t nc,
                      const double* affine) {
  if (!c || !dev_fields) return fail(MCLBM_EINVAL, "load_fields: NULL cavity or fields");
  // A batch steps all members with one parity; a loaded state is in the
  // even-step layout, so a member may be loaded only at an even batch step.
  if (c->in_batch && (!c->batch_clock || (*c->batch_clock & 1)))
    return fail(MCLBM_ESTATE, "load_fields: the batch is at an odd step; step it once more first");
  if (nc != 4 && nc != 5) return fail(MCLBM_EINVAL, "load_fields: nc must be 4 or 5");
  if (c->P.nl != 3) return fail(MCLBM_EUNSUPPORTED, "load_fields: one thermal lattice only");
  if (sx < 1 || sy < 1 || (long long)sx * sy > (1LL << 30))
    return fail(MCLBM_EINVAL, "load_fields: source grid must be at least 1 x 1 and at most 2^30 cells");
  if (affine)
    for (int q = 0; q < 2 * nc; ++q)
      if (!std::isfinite(affine[q])) return fail(MCLBM_EINVAL, "load_fields: affine map not finite");
  return enqueue_load_fields(c, dev_fields, sx, sy, nc, affine);
}

int mclbm_copy_state(mclbm_cavity* dst, const mclbm_cavity* src) {
  if (!dst || !src || dst == src) return fail(MCLBM_EINVAL, "copy_state: NULL or identical cavities");
  mclbm_config a = dst->cfg, b = src->cfg;
  a.storage = b.storage = MCLBM_FP32S;
  if (config_key(a) != config_key(b))
    return fail(MCLBM_EINVAL, "copy_state: the configurations differ beyond storage and launch shape");
  if (dst->L.plane != src->L.plane)
    return fail(MCLBM_EINVAL, "copy_state: the population planes differ in pitch (MCLBM_PLANE_PAD)");
  if (src->t & 1) return fail(MCLBM_ESTATE, "copy_state: the source is at an odd step; step it once more");
  if (dst->in_batch && (!dst->batch_clock || (*dst->batch_clock & 1)))
    return fail(MCLBM_ESTATE, "copy_state: the destination's batch is at an odd step");
  HIP_TRY(hipStreamSynchronize(src->stream));
  const long long n = 9LL * dst->P.nl * dst->L.plane;
  int rc;
  switch (src->cfg.storage) {
    case MCLBM_FP32S: rc = launch_convert<StorF32<false>>(dst, src, n); break;
    case MCLBM_FP16S: rc = launch_convert<StorF16<false>>(dst, src, n); break;
    default: rc = launch_convert<StorBF16<false>>(dst, src, n);
  }
  if (rc) return rc;
  mclbm_cavity* s_ = const_cast<mclbm_cavity*>(src);
  for (int k = 0; k < 2; ++k)
    HIP_TRY(hipMemcpyAsync(dst->d2(k), s_->d2(k), (size_t)dst->L.plane * sizeof(float2),
                           hipMemcpyDeviceToDevice, dst->stream));
  HIP_TRY(hipMemcpyAsync(dst->d5(), s_->d5(), (size_t)6 * (dst->P.nl - 2) * dst->L.px * sizeof(float),
                         hipMemcpyDeviceToDevice, dst->stream));
  HIP_TRY(hipMemcpyAsync(dst->snap(), s_->snap(), (size_t)3 * dst->cfg.nx * dst->cfg.ny * sizeof(double),
                         hipMemcpyDeviceToDevice, dst->stream));
  HIP_TRY(hipStreamSynchronize(dst->stream));
  dst->t = src->t;
  ++dst->epoch;
  return MCLBM_OK;
}

int mclbm_step(mclbm_cavity* c, int64_t nsteps) {
  if (!c) return fail(MCLBM_EINVAL, "cavity is NULL");
  if (c->in_batch) return fail(MCLBM_ESTATE, "cavity belongs to a batch: use the batch calls");
  if (nsteps < 0) return fail(MCLBM_EINVAL, "nsteps must be >= 0");
  const int64_t every = c->nu_every;
  return dispatch(c, [&](auto k) {
    for (int64_t s = 0; s < nsteps;) {
      // a pair of steps keeps its odd step in registers: where a record
      // falls on that odd step, the pair is run as two single steps
      const bool split = every > 0 && (c->t + 1) % every == 0;
      if (c->two && (c->t & 1) == 0 && nsteps - s >= 2 && !split) {
        int rc = launch_step2<decltype(k)>(c);
        if (rc) return rc;
        c->t += 2;
        s += 2;
      } else {
        int rc = launch_step<decltype(k)>(c);
        if (rc) return rc;
        c->t += 1;
        s += 1;
      }
      if (every > 0 && c->t % every == 0) {
        int rc = launch_nusselt(c, c->nu_ring + 4 * (c->nu_count % c->nu_cap));
        if (rc) return rc;
        ++c->nu_count;
      }
    }
    return (int)MCLBM_OK;
  });
}

int mclbm_record_nusselt(mclbm_cavity* c, int32_t every, double* dev_ring, int32_t capacity) {
  if (!c) return fail(MCLBM_EINVAL, "cavity is NULL");
  if (c->in_batch) return fail(MCLBM_ESTATE, "cavity belongs to a batch: use the batch calls");
  if (every < 0) return fail(MCLBM_EINVAL, "record_nusselt: every must be >= 0");
  if (every > 0 && (!dev_ring || capacity < 1 || reinterpret_cast<uintptr_t>(dev_ring) % alignof(double) != 0))
    return fail(MCLBM_EINVAL, "record_nusselt: needs an aligned device ring of capacity >= 1");
  c->nu_every = every;
  c->nu_ring = every > 0 ? dev_ring : nullptr;
  c->nu_cap = every > 0 ? capacity : 0;
  c->nu_count = 0;
  return MCLBM_OK;
}

int64_t mclbm_nusselt_records(const mclbm_cavity* c) { return c ? c->nu_count : -1; }

int64_t mclbm_time(const mclbm_cavity* c) { return c ? c->t : -1; }

int mclbm_export_moments(mclbm_cavity* c, uint32_t mask, double* dev_out, size_t n_doubles) {
  if (!c || !dev_out) return fail(MCLBM_EINVAL, "NULL argument");
  if (mask == 0 || mask > MCLBM_FIELD_MASK) return fail(MCLBM_EINVAL, "bad field mask");
  const long long nn = (long long)c->cfg.nx * c->cfg.ny;
  const int nf = __builtin_popcount(mask);
  if (n_doubles < (size_t)nf * nn) return fail(MCLBM_EINVAL, "output too small");
  const double rf = (double)c->P.rho_f_ref, rp = (double)c->P.rho_p_ref;
  const double invR = 1.0 / c->D.v[MCLBM_D_R];
  return dispatch(c, [&](auto k) {
    using S = typename decltype(k)::S;
    using I = typename decltype(k)::I;
    const auto* pop = reinterpret_cast<const typename S::T*>(c->pop());
    if (c->t & 1)
      k_export<true, S, I, decltype(k)::NL><<<node_blocks(c), 256, 0, c->stream>>>(c->P, pop, c->d5(), rf, rp, invR, mask, dev_out);
    else
      k_export<false, S, I, decltype(k)::NL><<<node_blocks(c), 256, 0, c->stream>>>(c->P, pop, c->d5(), rf, rp, invR, mask, dev_out);
    return launch_check("k_export");
  });
}

int mclbm_read_moments(mclbm_cavity* c, uint32_t mask, double* host_out, size_t n_doubles) {
  if (!c || !host_out) return fail(MCLBM_EINVAL, "NULL argument");
  if (mask == 0 || mask > MCLBM_FIELD_MASK) return fail(MCLBM_EINVAL, "bad field mask");
  const long long nn = (long long)c->cfg.nx * c->cfg.ny;
  if (n_doubles < (size_t)__builtin_popcount(mask) * nn) return fail(MCLBM_EINVAL, "output too small");
  int slot = 0;
  for (int b = 0; b < MCLBM_FIELD_COUNT; ++b) {
    if (!((mask >> b) & 1u)) continue;
    int rc = mclbm_export_moments(c, 1u << b, c->stage(), (size_t)nn);
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(host_out + (size_t)slot * nn, c->stage(), (size_t)nn * sizeof(double),
                           hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    ++slot;
  }
  return MCLBM_OK;
}


int mclbm_export_populations(mclbm_cavity* c, double* dev_out, size_t n_doubles) {
  if (!c || !dev_out) return fail(MCLBM_EINVAL, "NULL argument");
  const long long nn = (long long)c->cfg.nx * c->cfg.ny;
  if (n_doubles < (size_t)9 * c->P.nl * nn) return fail(MCLBM_EINVAL, "output too small");
  return export_pops(c, -1, dev_out);
}

int mclbm_read_populations(mclbm_cavity* c, double* host_out, size_t n_doubles) {
  if (!c || !host_out) return fail(MCLBM_EINVAL, "NULL argument");
  const long long nn = (long long)c->cfg.nx * c->cfg.ny;
  if (n_doubles < (size_t)9 * c->P.nl * nn) return fail(MCLBM_EINVAL, "output too small");
  for (int q = 0; q < 9 * c->P.nl; ++q) {  // one plane at a time through the stage
    int rc = export_pops(c, q, c->stage());
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(host_out + (size_t)q * nn, c->stage(), (size_t)nn * sizeof(double),
                           hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
  }
  return MCLBM_OK;
}

int mclbm_nusselt(mclbm_cavity* c, double* nu_hot, double* nu_cold, double* nu_hot_k) {
  if (!c) return fail(MCLBM_EINVAL, "cavity is NULL");
  double h[4];
  int rc = enqueue_nusselt(c, h);
  if (rc) return rc;
  HIP_TRY(hipStreamSynchronize(c->stream));
  return finish_nusselt(h, nu_hot, nu_cold, nu_hot_k);
}

int mclbm_residual(mclbm_cavity* c, double* res_u, double* res_theta) {
  if (!c) return fail(MCLBM_EINVAL, "cavity is NULL");
  double h[5];
  int rc = enqueue_residual(c, h);
  if (rc) return rc;
  HIP_TRY(hipStreamSynchronize(c->stream));
  return finish_residual(h, res_u, res_theta);
}

int mclbm_residual_noalloc(mclbm_cavity* c, double* dev_out) {
  if (!c) return fail(MCLBM_EINVAL, "cavity is NULL");
  if (!dev_out || reinterpret_cast<uintptr_t>(dev_out) % alignof(double) != 0)
    return fail(MCLBM_EINVAL, "dev_out must be a non-NULL device pointer aligned to 8 bytes");
  const size_t need = (size_t)5 * c->L.red_blocks * sizeof(double);
  if (need > (size_t)MCLBM_NOALLOC_SCRATCH_BYTES)
    return fail(MCLBM_EINVAL, "cavity of " + std::to_string((long long)c->cfg.nx * c->cfg.ny) +
                                  " nodes exceeds the static scratch of mclbm_residual_noalloc (at most " +
                                  std::to_string((long long)MCLBM_NOALLOC_MAX_NODES) + " nodes)");
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != c->device) return fail(MCLBM_EINVAL, "the cavity's device must be current");
  double* part = nullptr;
  int rc = noalloc_scratch(dev, &part);
  if (rc) return rc;
  rc = enqueue_residual_partials(c, part);
  if (rc) return rc;
  k_sum_partials_finish<<<1, 256, 0, c->stream>>>(part, c->L.red_blocks, dev_out);
  return launch_check("k_sum_partials_finish");
}

int mclbm_derived(const mclbm_cavity* c, double* out, int n) {
  if (!c || !out || n < MCLBM_D_COUNT) return fail(MCLBM_EINVAL, "bad arguments");
  std::memcpy(out, c->D.v, sizeof(c->D.v));
  return MCLBM_OK;
}

int mclbm_checkpoint(mclbm_cavity* c, const char* path) {
  if (!c || !path) return fail(MCLBM_EINVAL, "checkpoint: NULL argument");
  HIP_TRY(hipStreamSynchronize(c->stream));
  const auto secs = ckpt_sections(c);
  std::string h = "{\"format\": \"mclbm-checkpoint\", \"version\": " + std::to_string(kCkptVersion) +
                  ", \"abi\": " + std::to_string(MCLBM_ABI_VERSION);
  char buf[256];
  const mclbm_config& g = c->cfg;
  std::snprintf(buf, sizeof buf, ", \"nx\": %d, \"ny\": %d, \"Ra\": %.17g, \"Pr\": %.17g, \"phi0\": %.17g, \"dp_m\": %.17g",
                g.nx, g.ny, g.Ra, g.Pr, g.phi0, g.dp_m);
  h += buf;
  std::snprintf(buf, sizeof buf, ", \"tau_f\": %.17g, \"force_mask\": %u, \"storage\": %d, \"lattices\": %d",
                g.tau_f, g.force_mask, g.storage, c->P.nl);
  h += buf;
  h += ", \"derived\": [";
  for (int k = 0; k < MCLBM_D_COUNT; ++k) {
    std::snprintf(buf, sizeof buf, "%s%.17g", k ? ", " : "", c->D.v[k]);
    h += buf;
  }
  h += "], \"t\": " + std::to_string((long long)c->t) + ", \"parity\": " + std::to_string((int)(c->t & 1));
  h += ", \"config_hex\": \"" + config_key(c->cfg) + "\"";
  h += ", \"xi_hex\": \"" + hex_of(c->xi.data(), c->xi.size() * sizeof(double)) + "\"";
  h += ", \"sections\": [";
  for (size_t k = 0; k < secs.size(); ++k)
    h += std::string(k ? ", " : "") + "{\"name\": \"" + secs[k].name + "\", \"bytes\": " + std::to_string(secs[k].bytes) + "}";
  h += "]}\n";
  FILE* fp = std::fopen(path, "wb");
  if (!fp) return fail(MCLBM_EINVAL, std::string("checkpoint: cannot open ") + path);
  bool ok = std::fwrite(h.data(), 1, h.size(), fp) == h.size();
  std::vector<char> host;
  for (const auto& sc : secs) {
    if (!ok) break;
    host.resize(sc.bytes);
    if (sc.bytes) {
      hipError_t e = ckpt_to_host(c, sc, host.data());
      if (e != hipSuccess) {
        std::fclose(fp);
        return hip_fail(e, "checkpoint: hipMemcpy");
      }
      ok = std::fwrite(host.data(), 1, sc.bytes, fp) == sc.bytes;
    }
  }
  ok = (std::fclose(fp) == 0) && ok;
  if (!ok) return fail(MCLBM_EINVAL, std::string("checkpoint: write failed: ") + path);
  return MCLBM_OK;
}

int mclbm_restore(mclbm_cavity* c, const char* path) {
  if (!c || !path) return fail(MCLBM_EINVAL, "restore: NULL argument");
  if (c->in_batch) return fail(MCLBM_ESTATE, "restore: cavity belongs to a batch");
  FILE* fp = std::fopen(path, "rb");
  if (!fp) return fail(MCLBM_EINVAL, std::string("restore: cannot open ") + path);
  CkptHeader H;
  const auto secs = ckpt_sections(c);
  auto bad = [&](const std::string& why) {
    std::fclose(fp);
    return fail(MCLBM_EINVAL, "restore: " + why);
  };
  if (read_ckpt_header(fp, H) != MCLBM_OK) return bad(mclbm_last_error());
  if (config_key(H.cfg) != config_key(c->cfg)) return bad("the configuration differs from the cavity's");
  if (H.xi.size() != c->xi.size() ||
      (!H.xi.empty() && std::memcmp(H.xi.data(), c->xi.data(), H.xi.size() * sizeof(double)) != 0))
    return bad("the initial perturbation field differs from the cavity's");
  const long long t = H.t;
  const std::string& h = H.line;
  for (const auto& sc : secs) {
    const std::string key = std::string("{\"name\": \"") + sc.name + "\", \"bytes\": " + std::to_string(sc.bytes) + "}";
    if (h.find(key) == std::string::npos) return bad(std::string("section size mismatch: ") + sc.name);
  }
  // read everything first, so that a short file leaves the cavity unchanged
  std::vector<std::vector<char>> data(secs.size());
  for (size_t k = 0; k < secs.size(); ++k) {
    data[k].resize(secs[k].bytes);
    if (secs[k].bytes && std::fread(data[k].data(), 1, secs[k].bytes, fp) != secs[k].bytes)
      return bad("file too short");
  }
  if (std::fgetc(fp) != EOF) return bad("trailing bytes");
  std::fclose(fp);
  HIP_TRY(hipStreamSynchronize(c->stream));
  for (size_t k = 0; k < secs.size(); ++k)
    if (secs[k].bytes) HIP_TRY(ckpt_to_device(c, secs[k], data[k].data()));
  c->t = t;
  ++c->epoch;
  return MCLBM_OK;
}

int mclbm_checkpoint_info(const char* path, mclbm_config* cfg_out, int64_t* t_out, double* xi_out,
                          size_t xi_cap, size_t* n_xi) {
  if (!path) return fail(MCLBM_EINVAL, "checkpoint_info: path is NULL");
  FILE* fp = std::fopen(path, "rb");
  if (!fp) return fail(MCLBM_EINVAL, std::string("checkpoint_info: cannot open ") + path);
  CkptHeader H;
  const int rc = read_ckpt_header(fp, H);
  std::fclose(fp);
  if (rc) return rc;
  if (xi_out && !H.xi.empty()) {
    if (xi_cap < H.xi.size()) return fail(MCLBM_EINVAL, "checkpoint_info: xi_out holds fewer than nx*ny values");
    std::memcpy(xi_out, H.xi.data(), H.xi.size() * sizeof(double));
  }
  if (cfg_out) *cfg_out = H.cfg;
  if (t_out) *t_out = (int64_t)H.t;
  if (n_xi) *n_xi = H.xi.size();
  return MCLBM_OK;
}

int mclbm_destroy(mclbm_cavity* c) {
  if (!c) return MCLBM_OK;
  if (c->in_batch) return fail(MCLBM_ESTATE, "cavity belongs to a batch: destroy the batch");
  hipError_t e = hipStreamSynchronize(c->stream);
  delete c;
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  return MCLBM_OK;
}

const char* mclbm_last_error(void) { return g_err.c_str(); }

int mclbm_copy_kernel(void* dst, const void* src, size_t bytes, void* stream) {
  if (!dst || !src || bytes % 16 != 0) return fail(MCLBM_EINVAL, "copy: bad arguments");
  const long long n = (long long)(bytes / 16);
  const long long blocks = (n + 256 * kCopyUnroll - 1) / (256 * kCopyUnroll);
  if (blocks > 2147483647LL) return fail(MCLBM_EINVAL, "copy: too large");
  if (blocks == 0) return MCLBM_OK;
  k_copy<<<(unsigned)blocks, 256, 0, reinterpret_cast<hipStream_t>(stream)>>>(
      reinterpret_cast<v4f*>(dst), reinterpret_cast<const v4f*>(src), n);
  return launch_check("k_copy");
}

const char* mclbm_version(void) { return "mclbm 0.1.0 (gfx950)"; }
int mclbm_abi_version(void) { return MCLBM_ABI_VERSION; }

}  // extern "C"

// ===========================================================================
// Batched sweeps (host side)
// ===========================================================================

struct mclbm_batch {
  int n = 0;
  std::vector<mclbm_cavity> cav;
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;  // private stream the step graph is captured on
  char* base = nullptr;
  size_t bytes = 0;
  size_t off_desc = 0, off_ntiles = 0, off_tiles = 0, off_ntiles2 = 0, off_tiles2 = 0;
  size_t off_red = 0, off_rlist = 0, off_rtiles = 0, off_rout = 0;
  int tile_cap = 0, tile_cap2 = 0, rtile_cap = 0;
  int nr = 0, nrt = 0;  // active cavities, (cavity, block) entries of the residual
  std::vector<int> host_rlist;
  std::vector<int2> host_rtiles;
  std::vector<RedDesc> host_red;
  std::vector<char> active;
  std::vector<CavDesc> host_desc;
  std::vector<int2> host_tiles, host_tiles2;
  int ntiles = 0, ntiles2 = 0;
  bool two = false;  // two steps per launch (k_step2_batch) from even steps
  bool percav = false;  // one workgroup per cavity for many steps (k_step_cavity)
  // pinned host results of the reductions: 16 doubles per listed active
  // cavity, then 16 per cavity for the inactive ones' Nusselt numbers
  double* h_red = nullptr;
  int flip = 0;      // two-step launches since the descriptors were written, mod 2
  int64_t t = 0;  // steps of the active cavities
  int storage = MCLBM_FP32S;
  bool nt = false, idx32 = true;
  unsigned grid = 0, grid2 = 0;
  int graph_steps = 32;
  hipGraphExec_t gexec = nullptr;
  int gexec_steps = 0;

  CavDesc* d_desc() { return reinterpret_cast<CavDesc*>(base + off_desc); }
  int* d_ntiles() { return reinterpret_cast<int*>(base + off_ntiles); }
  int2* d_tiles() { return reinterpret_cast<int2*>(base + off_tiles); }
  int* d_ntiles2() { return reinterpret_cast<int*>(base + off_ntiles2); }
  int2* d_tiles2() { return reinterpret_cast<int2*>(base + off_tiles2); }
  RedDesc* d_red() { return reinterpret_cast<RedDesc*>(base + off_red); }
  int* d_rlist() { return reinterpret_cast<int*>(base + off_rlist); }
  int2* d_rtiles() { return reinterpret_cast<int2*>(base + off_rtiles); }
  double* d_rout() { return reinterpret_cast<double*>(base + off_rout); }
  double* h_inactive(int k) { return h_red + 16 * (size_t)n + 16 * (size_t)k; }
  // the Nusselt numbers of a dropped cavity in h_inactive(k) were computed
  // at step nu_t[k] of state epoch nu_epoch[k] (-1: none); a dropped cavity
  // is not stepped, so they stay valid until either changes
  std::vector<int64_t> nu_t;
  std::vector<uint64_t> nu_epoch;
};

namespace {

constexpr int kShapes[4][2] = {{256, 1}, {128, 2}, {64, 4}, {32, 8}};

int tiles_of(int nx, int ny, int bx, int by) { return ((nx + bx - 1) / bx) * ((ny + by - 1) / by); }

struct BatchLayout {
  size_t off_desc, off_ntiles, off_tiles, off_ntiles2, off_tiles2, total;
  size_t off_red, off_rlist, off_rtiles, off_rout;
  int tile_cap, tile_cap2, rtile_cap;
  bool two;
  bool pad;  // members' planes padded: the batch's working set streams from HBM
  std::vector<size_t> off_cav;
};

// A cavity's configuration inside a batch: the batch's schedule written
// into steps_per_launch (which the checkpoint key leaves out).
mclbm_config member_config(const mclbm_config& c, bool two) {
  mclbm_config m = c;
  m.steps_per_launch = two ? 2 : 1;
  return m;
}

// band heights the autotuner tries for two-step batches
constexpr int kBands2[4] = {3, 4, 6, 8};

// two-step tiles of a cavity at the lowest band the batch may use
int tiles2_of(const mclbm_config& c) {
  const int band = std::min(kBands2[0], band2_of(c));
  return strips2_of(c) * ((c.ny + band - 1) / band);
}

int batch_layout(const mclbm_config* cfgs, int n, BatchLayout& B) {
  if (!cfgs || n < 1) return fail(MCLBM_EINVAL, "batch needs n >= 1 configurations");
  long long cap = 0, cap2 = 0, nodes = 0, rcap = 0;
  int n1 = 0, n2 = 0;    // cavities asking for one or for two steps per launch
  bool possible = true;  // every cavity can take two steps per launch
  double used = 0.0;     // nodes weighted by the share of strip lanes they fill
  double streaming = 0.0;  // FP32 population and lag-field bytes of all members
  for (int k = 0; k < n; ++k) {
    int rc = validate(&cfgs[k]);
    if (rc) return fail(rc, "cavity " + std::to_string(k) + ": " + g_err);
    if (cfgs[k].storage != cfgs[0].storage) return fail(MCLBM_EINVAL, "all cavities of a batch share the storage type");
    if (cfgs[k].thermal_lattices == 2)
      return fail(MCLBM_EUNSUPPORTED, "cavity " + std::to_string(k) + ": batches take one thermal lattice");
    n1 += cfgs[k].steps_per_launch == 1;
    n2 += cfgs[k].steps_per_launch == 2;
    possible = possible && two_step_batchable(cfgs[k]) && cfgs[k].storage == MCLBM_FP32S;
    if (cfgs[k].steps_per_launch == 2 && !two_step_batchable(cfgs[k]))
      return fail(MCLBM_EUNSUPPORTED,
                  "cavity " + std::to_string(k) + ": two steps per launch in a batch need populations below 2 GiB");
    const long long nn = (long long)cfgs[k].nx * cfgs[k].ny;
    nodes += nn;
    used += (double)nn * cfgs[k].nx / (double)(kStrip2 * strips2_of(cfgs[k]));
    streaming += (double)((cfgs[k].nx + 63) / 64 * 64) * cfgs[k].ny * (27 * 4 + 2 * 8);
    int m = 0;
    for (const auto& sh : kShapes) m = std::max(m, tiles_of(cfgs[k].nx, cfgs[k].ny, sh[0], sh[1]));
    cap += m;
    rcap += (nn + 255) / 256;
  }
  if (n2 != 0 && n2 != n)
    return fail(MCLBM_EUNSUPPORTED,
                "a batch runs every cavity one step per launch, or every cavity two (steps_per_launch 2 for all)");
  if (cap > (1LL << 30) || rcap > (1LL << 30)) return fail(MCLBM_EINVAL, "batch too large");
  B.rtile_cap = (int)rcap;
  // Members of a batch whose working set streams from HBM (counted in FP32,
  // so that batches of one set of cavities in different storage types lay
  // them out alike) pad their planes like single cavities from 2^20 nodes:
  // the 256-cavity sweep (64^2 to 512^2 members, 6 GB) +3 % with two steps
  // per launch.
  B.pad = streaming > (double)kStreamingBytes;
  // Automatic (every cavity 0): two steps per launch for FP32 batches from
  // 2^20 nodes whose cavities fill at least 60 % of their strips' lanes
  // (measured: 1.06-1.51x from 1 M to 17 M nodes of 128- to 512-column
  // cavities; slower below 2^20 nodes and for 64-column cavities, which
  // leave most of a second strip idle).
  B.two = n2 == n || (n1 == 0 && n2 == 0 && possible && nodes >= (1LL << 20) && used >= 0.6 * (double)nodes);
  if (B.two)
    for (int k = 0; k < n; ++k) cap2 += tiles2_of(cfgs[k]);
  if (cap2 > (1LL << 30)) return fail(MCLBM_EINVAL, "batch too large");
  B.tile_cap = (int)(8 * ((cap + 7) / 8) + 8);
  B.tile_cap2 = B.two ? (int)(8 * ((cap2 + 7) / 8) + 8) : 0;
  size_t off = 0;
  B.off_desc = off;
  off = align_up(off + (size_t)n * sizeof(CavDesc));
  B.off_ntiles = off;
  off = align_up(off + sizeof(int));
  B.off_tiles = off;
  off = align_up(off + (size_t)B.tile_cap * sizeof(int2));
  B.off_ntiles2 = off;
  off = align_up(off + sizeof(int));
  B.off_tiles2 = off;
  off = align_up(off + (size_t)B.tile_cap2 * sizeof(int2));
  B.off_red = off;
  off = align_up(off + (size_t)n * sizeof(RedDesc));
  B.off_rlist = off;
  off = align_up(off + (size_t)n * sizeof(int));
  B.off_rtiles = off;
  off = align_up(off + (size_t)B.rtile_cap * sizeof(int2));
  B.off_rout = off;
  off = align_up(off + (size_t)16 * n * sizeof(double));
  B.off_cav.resize(n);
  for (int k = 0; k < n; ++k) {
    B.off_cav[k] = off;
    off = align_up(off + make_layout(member_config(cfgs[k], B.two), true, B.pad).total);
  }
  B.total = off;
  return MCLBM_OK;
}

CavDesc make_desc(mclbm_cavity* c) {
  CavDesc d{};
  d.P = c->P;
  d.pop[0] = c->pop();
  d.pop[1] = c->two ? c->pop_other() : c->pop();
  d.d2[0] = c->d2(0);
  d.d2[1] = c->d2(1);
  d.d5 = c->d5();
  d.bx = (int)c->block.x;
  d.by = (int)c->block.y;
  d.tiles_x = c->tiles_x;
  d.strips2 = c->strips2;
  d.band2 = c->band2;
  return d;
}

// Tile table: the tiles of the active cavities (cavity-major, row-major
// within a cavity) cut into 8 contiguous chunks; chunk j takes entries
// j, j + 8, j + 16, ... so that the workgroups one XCD receives (b = j mod 8
// under round-robin dealing) sweep one contiguous band.  Then uploaded with
// the descriptors.  Sync.
void deal_to_xcds(const std::vector<int2>& list, std::vector<int2>& table) {
  const int L = (int)list.size();
  const int m = (L + 7) / 8;
  table.assign((size_t)8 * m, make_int2(-1, 0));
  for (int j = 0; j < 8; ++j)
    for (int q = 0; q < m; ++q) {
      const int src = j * m + q;
      if (src < L) table[(size_t)8 * q + j] = list[src];
    }
}

// The dispatch order of band_of_tile, for the batch's tile table.
int band_slot(int slot, int segs, int mix) {
  const int w = mix * kBandWindow;
  if (mix <= 1 || slot >= segs / w * w) return slot;
  const int i = slot % w;
  return slot - i + (i % mix) * kBandWindow + i / mix;
}

// With two steps per launch, the (strip, band) tiles of each active cavity
// (band-row-major, the band rows in the cavity's interleaved dispatch order,
// band_slot) form the second table, dealt to the XCDs the same way.
// The descriptors take the current roles of the copies: flip restarts at 0.
int upload_tables(mclbm_batch* b) {
  std::vector<int2> list, list2;
  for (int k = 0; k < b->n; ++k) {
    if (b->cav[k].block.x * b->cav[k].block.y != 256)
      return fail(MCLBM_EINVAL, "batched tiles must cover 256 nodes");
    if (!b->active[k]) continue;
    const int nt = tiles_of(b->cav[k].cfg.nx, b->cav[k].cfg.ny, b->cav[k].block.x, b->cav[k].block.y);
    for (int t = 0; t < nt; ++t) list.push_back(make_int2(k, t));
    if (b->two) {
      const mclbm_cavity& c = b->cav[k];
      const int segs = (c.cfg.ny + c.band2 - 1) / c.band2;
      for (int slot = 0; slot < segs; ++slot) {
        const int seg = band_slot(slot, segs, c.mix2);
        for (int st = 0; st < c.strips2; ++st) list2.push_back(make_int2(k, seg * c.strips2 + st));
      }
    }
  }
  deal_to_xcds(list, b->host_tiles);
  b->ntiles = (int)b->host_tiles.size();
  if (b->ntiles > b->tile_cap) return fail(MCLBM_EINVAL, "tile table overflow");
  deal_to_xcds(list2, b->host_tiles2);
  b->ntiles2 = (int)b->host_tiles2.size();
  if (b->ntiles2 > b->tile_cap2) return fail(MCLBM_EINVAL, "two-step tile table overflow");
  b->host_desc.resize(b->n);
  for (int k = 0; k < b->n; ++k) b->host_desc[k] = make_desc(&b->cav[k]);
  // reductions: the active cavities, and their (cavity, block) entries
  b->host_red.resize(b->n);
  b->host_rlist.clear();
  b->host_rtiles.clear();
  for (int k = 0; k < b->n; ++k) {
    mclbm_cavity* c = &b->cav[k];
    RedDesc& r = b->host_red[k];
    r.snap = c->snap();
    r.part = c->part();
    r.rho_f_ref = (double)c->P.rho_f_ref;
    r.rho_p_ref = (double)c->P.rho_p_ref;
    r.R = c->D.v[MCLBM_D_R];
    r.Ck = c->D.v[MCLBM_D_CK];
    r.red_blocks = c->L.red_blocks;
    r.pad = 0;
    if (!b->active[k]) continue;
    b->host_rlist.push_back(k);
    for (int q = 0; q < c->L.red_blocks; ++q) b->host_rtiles.push_back(make_int2(k, q));
  }
  b->nr = (int)b->host_rlist.size();
  b->nrt = (int)b->host_rtiles.size();
  if (b->nrt > b->rtile_cap) return fail(MCLBM_EINVAL, "reduction table overflow");
  HIP_TRY(hipMemcpyAsync(b->d_red(), b->host_red.data(), b->host_red.size() * sizeof(RedDesc),
                         hipMemcpyHostToDevice, b->stream));
  if (b->nr > 0) {
    HIP_TRY(hipMemcpyAsync(b->d_rlist(), b->host_rlist.data(), (size_t)b->nr * sizeof(int),
                           hipMemcpyHostToDevice, b->stream));
    HIP_TRY(hipMemcpyAsync(b->d_rtiles(), b->host_rtiles.data(), (size_t)b->nrt * sizeof(int2),
                           hipMemcpyHostToDevice, b->stream));
  }
  HIP_TRY(hipMemcpyAsync(b->d_desc(), b->host_desc.data(), b->host_desc.size() * sizeof(CavDesc),
                         hipMemcpyHostToDevice, b->stream));
  if (b->ntiles > 0)
    HIP_TRY(hipMemcpyAsync(b->d_tiles(), b->host_tiles.data(), (size_t)b->ntiles * sizeof(int2),
                           hipMemcpyHostToDevice, b->stream));
  HIP_TRY(hipMemcpyAsync(b->d_ntiles(), &b->ntiles, sizeof(int), hipMemcpyHostToDevice, b->stream));
  if (b->two) {
    if (b->ntiles2 > 0)
      HIP_TRY(hipMemcpyAsync(b->d_tiles2(), b->host_tiles2.data(), (size_t)b->ntiles2 * sizeof(int2),
                             hipMemcpyHostToDevice, b->stream));
    HIP_TRY(hipMemcpyAsync(b->d_ntiles2(), &b->ntiles2, sizeof(int), hipMemcpyHostToDevice, b->stream));
  }
  HIP_TRY(hipStreamSynchronize(b->stream));
  b->flip = 0;
  return MCLBM_OK;
}

template <class K>
void batch_launch(mclbm_batch* b, hipStream_t s, bool odd, int flip) {
  using I = typename K::I;
  if (!odd)
    k_step_batch<false, typename K::SE, I><<<b->grid, 256, 0, s>>>(b->d_desc(), b->d_tiles(), b->d_ntiles(), flip);
  else
    k_step_batch<true, typename K::SO, I><<<b->grid, 256, 0, s>>>(b->d_desc(), b->d_tiles(), b->d_ntiles(), flip);
}

// Two steps (even, odd) of every active cavity; cached access at every size,
// as for a single cavity.
template <class K>
int batch_launch2(mclbm_batch* b, hipStream_t s, int flip) {
  if constexpr (sizeof(typename K::I) == 4) {
    k_step2_batch<typename K::S><<<b->grid2, 64, 0, s>>>(b->d_desc(), b->d_tiles2(), b->d_ntiles2(), flip);
    return MCLBM_OK;
  } else {
    return fail(MCLBM_EUNSUPPORTED, "two steps per launch: 32-bit offsets only");
  }
}

// One workgroup per active cavity, `steps` (even) steps per launch.
constexpr int64_t kPerCavChunk = 256;  // steps per launch

bool percav_eligible(const mclbm_batch* b) {
  if (b->two || !b->idx32 || b->nt) return false;
  for (int k = 0; k < b->n; ++k)
    if ((long long)b->cav[k].cfg.nx * b->cav[k].cfg.ny > kPerCavNodes) return false;
  return true;
}

// The default schedule: one workgroup per cavity when the cavities are
// small (at most 64^2) and about as many as compute units or more (measured
// faster from 128 cavities of 32^2 and 256 of 64^2; slower with 16 of 32^2,
// 64 of 64^2 or 16 of 128^2).
bool percav_default(const mclbm_batch* b) {
  if (!percav_eligible(b)) return false;
  long long most = 0;
  for (int k = 0; k < b->n; ++k) most = std::max(most, (long long)b->cav[k].cfg.nx * b->cav[k].cfg.ny);
  if (most > 64 * 64) return false;
  return (long long)b->n >= std::max(128LL, 256LL * most / (64 * 64));
}

void batch_advance(mclbm_batch* b, int64_t k) {
  b->t += k;
  for (int c = 0; c < b->n; ++c)
    if (b->active[c]) b->cav[c].t += k;
}

// after `launches` two-step launches: the copies and lag fields of every
// active cavity have swapped roles that many times
void batch_advance2(mclbm_batch* b, int64_t launches) {
  batch_advance(b, 2 * launches);
  if (launches & 1) {
    for (int c = 0; c < b->n; ++c)
      if (b->active[c]) {
        b->cav[c].popsel ^= 1;
        b->cav[c].d2sel ^= 1;
      }
    b->flip ^= 1;
  }
}

int batch_direct_step(mclbm_batch* b) {
  int rc = dispatch_kinds(b->storage, b->idx32, b->nt, [&](auto k) {
    batch_launch<decltype(k)>(b, b->stream, (b->t & 1) != 0, b->flip);
    return launch_check("k_step_batch");
  });
  if (rc) return rc;
  batch_advance(b, 1);
  return MCLBM_OK;
}

int batch_direct_step2(mclbm_batch* b) {
  int rc = dispatch_kinds(b->storage, b->idx32, b->nt, [&](auto k) {
    int r = batch_launch2<decltype(k)>(b, b->stream, b->flip);
    if (r) return r;
    return launch_check("k_step2_batch");
  });
  if (rc) return rc;
  batch_advance2(b, 1);
  return MCLBM_OK;
}

// `steps` (even) steps of every active cavity from an even step, one
// workgroup per cavity.
int batch_cavity_steps(mclbm_batch* b, int64_t steps) {
  if (b->nr > 0) {
    int rc = dispatch_kinds(b->storage, b->idx32, b->nt, [&](auto k) {
      using K = decltype(k);
      if constexpr (sizeof(typename K::I) == 4 && std::is_same_v<typename K::SE, typename K::S>) {
        k_step_cavity<typename K::SE, typename K::SO, typename K::I>
            <<<b->nr, kPerCavThreads, 0, b->stream>>>(b->d_desc(), b->d_rlist(), (int)steps);
        return launch_check("k_step_cavity");
      } else {
        return fail(MCLBM_EUNSUPPORTED, "one workgroup per cavity: small cavities only");
      }
    });
    if (rc) return rc;
  }
  batch_advance(b, steps);
  return MCLBM_OK;
}

// launches in one replay of the step graph
int graph_launches(const mclbm_batch* b) { return b->two ? b->graph_steps / 2 : b->graph_steps; }

void drop_graph(mclbm_batch* b) {
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  b->gexec = nullptr;
  b->gexec_steps = 0;
}

// Capture graph_steps launches (even, odd, even, ...) on the private
// stream, or graph_steps / 2 two-step launches with flip 0, 1, 0, ...; the
// graph is replayed on the batch's stream, from even steps and (two steps
// per launch) descriptors written with flip 0.
int capture_graph(mclbm_batch* b) {
  drop_graph(b);
  HIP_TRY(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
  int rc = dispatch_kinds(b->storage, b->idx32, b->nt, [&](auto k) {
    for (int q = 0; q < graph_launches(b); ++q) {
      if (b->two) {
        int r = batch_launch2<decltype(k)>(b, b->cap_stream, q & 1);
        if (r) return r;
      } else {
        batch_launch<decltype(k)>(b, b->cap_stream, (q & 1) != 0, 0);
      }
    }
    return (int)MCLBM_OK;
  });
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  e = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    b->gexec = nullptr;
    return hip_fail(e, "hipGraphInstantiate");
  }
  b->gexec_steps = b->graph_steps;
  return MCLBM_OK;
}

int batch_reset_all(mclbm_batch* b) {
  for (int k = 0; k < b->n; ++k) {
    int rc = enqueue_init(&b->cav[k]);
    if (rc) return rc;
    b->active[k] = 1;
  }
  b->t = 0;
  return upload_tables(b);
}

}  // namespace

extern "C" {

size_t mclbm_batch_device_bytes(const mclbm_config* cfgs, int32_t n) {
  BatchLayout B;
  if (batch_layout(cfgs, n, B)) return 0;
  return B.total;
}

int mclbm_batch_create(const mclbm_config* cfgs, int32_t n, const double* const* xis, void* dev_buf,
                       size_t bytes, void* stream, mclbm_batch** out) {
  if (!out) return fail(MCLBM_EINVAL, "out is NULL");
  *out = nullptr;
  BatchLayout B;
  int rc = batch_layout(cfgs, n, B);
  if (rc) return rc;
  if (!dev_buf) return fail(MCLBM_EINVAL, "dev_buf is NULL");
  if (reinterpret_cast<uintptr_t>(dev_buf) % kAlign != 0) return fail(MCLBM_EINVAL, "dev_buf must be 256-byte aligned");
  if (bytes < B.total) return fail(MCLBM_ENOMEM, "device buffer too small: need " + std::to_string(B.total) + " bytes");
  mclbm_batch* b = new (std::nothrow) mclbm_batch();
  if (!b) return fail(MCLBM_ENOMEM, "host allocation failed");
  b->n = n;
  b->stream = reinterpret_cast<hipStream_t>(stream);
  b->base = reinterpret_cast<char*>(dev_buf);
  b->bytes = bytes;
  b->off_desc = B.off_desc;
  b->off_ntiles = B.off_ntiles;
  b->off_tiles = B.off_tiles;
  b->tile_cap = B.tile_cap;
  b->off_ntiles2 = B.off_ntiles2;
  b->off_tiles2 = B.off_tiles2;
  b->tile_cap2 = B.tile_cap2;
  b->off_red = B.off_red;
  b->off_rlist = B.off_rlist;
  b->off_rtiles = B.off_rtiles;
  b->off_rout = B.off_rout;
  b->rtile_cap = B.rtile_cap;
  b->two = B.two;
  b->storage = cfgs[0].storage;
  b->cav.resize(n);
  b->active.assign(n, 1);
  size_t work = 0;
  bool idx32 = true;
  for (int k = 0; k < n; ++k) {
    mclbm_cavity* c = &b->cav[k];
    c->cfg = member_config(cfgs[k], B.two);
    if (xis && xis[k]) c->xi.assign(xis[k], xis[k] + (size_t)cfgs[k].nx * cfgs[k].ny);
    c->stream = b->stream;
    c->base = b->base + B.off_cav[k];
    c->pad_planes = B.pad;
    c->bytes = make_layout(c->cfg, true, B.pad).total;
    c->in_batch = true;
    c->batch_clock = &b->t;
    setup_cavity(c);
    setup_device(c);
    // the batched kernel runs 256-thread workgroups: every tile shape must
    // cover exactly 256 nodes (bx * by == 256)
    if (c->block.x * c->block.y != 256) {
      const int bx = cfgs[k].nx >= 256 ? 256 : (cfgs[k].nx >= 128 ? 128 : 64);
      c->block = dim3(bx, 256 / bx, 1);
      c->tiles_x = (cfgs[k].nx + bx - 1) / bx;
    }
    work += (size_t)27 * c->L.plane * storage_bytes(b->storage) + (size_t)2 * c->L.plane * sizeof(float2);
    idx32 = idx32 && c->idx32;
  }
  // one access policy for the whole launch, from the working set of the batch
  b->nt = work > kStreamingBytes;
  b->idx32 = idx32;
  for (int k = 0; k < n; ++k) {
    b->cav[k].nt = b->nt;
    b->cav[k].idx32 = b->idx32;
  }
  int dev = 0, ncu = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) ncu = v;
  }
  // One workgroup per table entry: a grid-stride loop over fewer, resident
  // workgroups measured 26 % slower on a 256-cavity sweep, because each
  // workgroup then waits on the dependent descriptor loads of every tile it
  // takes in turn; separate workgroups overlap them.
  (void)ncu;
  b->grid = (unsigned)B.tile_cap;
  b->grid2 = (unsigned)B.tile_cap2;
  b->percav = percav_default(b);
  hipError_t e = hipHostMalloc((void**)&b->h_red, (size_t)32 * n * sizeof(double), hipHostMallocDefault);
  if (e != hipSuccess) {
    b->h_red = nullptr;
    delete b;
    return hip_fail(e, "hipHostMalloc");
  }
  e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    (void)hipHostFree(b->h_red);
    delete b;
    return hip_fail(e, "hipStreamCreateWithFlags");
  }
  rc = batch_reset_all(b);
  if (rc) {
    (void)hipStreamDestroy(b->cap_stream);
    (void)hipHostFree(b->h_red);
    delete b;
    return rc;
  }
  *out = b;
  return MCLBM_OK;
}

int mclbm_batch_step(mclbm_batch* b, int64_t nsteps) {
  if (!b) return fail(MCLBM_EINVAL, "batch is NULL");
  if (nsteps < 0) return fail(MCLBM_EINVAL, "nsteps must be >= 0");
  bool any = false;
  for (int k = 0; k < b->n; ++k) any = any || b->active[k];
  if (!any) return MCLBM_OK;
  while (nsteps > 0) {
    if (b->percav && nsteps >= 2 && (b->t & 1) == 0) {
      const int64_t k = std::min<int64_t>(nsteps & ~int64_t(1), kPerCavChunk);
      int rc = batch_cavity_steps(b, k);
      if (rc) return rc;
      nsteps -= k;
    } else if (b->graph_steps > 0 && nsteps >= b->graph_steps && (b->t & 1) == 0) {
      if (b->flip) {
        // the graph was captured for descriptors written with flip 0
        int rc = upload_tables(b);
        if (rc) return rc;
      }
      if (!b->gexec || b->gexec_steps != b->graph_steps) {
        int rc = capture_graph(b);
        if (rc) return rc;
      }
      HIP_TRY(hipGraphLaunch(b->gexec, b->stream));
      if (b->two)
        batch_advance2(b, graph_launches(b));
      else
        batch_advance(b, b->graph_steps);
      nsteps -= b->graph_steps;
    } else if (b->two && nsteps >= 2 && (b->t & 1) == 0) {
      int rc = batch_direct_step2(b);
      if (rc) return rc;
      nsteps -= 2;
    } else {
      int rc = batch_direct_step(b);
      if (rc) return rc;
      nsteps -= 1;
    }
  }
  return MCLBM_OK;
}

int mclbm_batch_set_per_cavity(mclbm_batch* b, int32_t on) {
  if (!b) return fail(MCLBM_EINVAL, "batch is NULL");
  if (on && !percav_eligible(b))
    return fail(MCLBM_EINVAL, "one workgroup per cavity needs one step per launch and cavities of at most " +
                                  std::to_string(kPerCavNodes) + " nodes");
  HIP_TRY(hipStreamSynchronize(b->stream));
  b->percav = on != 0;
  return MCLBM_OK;
}

int32_t mclbm_batch_per_cavity(const mclbm_batch* b) { return b ? (b->percav ? 1 : 0) : -1; }

int mclbm_batch_set_graph_steps(mclbm_batch* b, int32_t steps) {
  if (!b) return fail(MCLBM_EINVAL, "batch is NULL");
  if (steps != 0 && (steps < 2 || (steps & 1))) return fail(MCLBM_EINVAL, "graph steps must be 0 or an even number >= 2");
  HIP_TRY(hipStreamSynchronize(b->stream));
  b->graph_steps = steps;
  drop_graph(b);
  return MCLBM_OK;
}

int mclbm_batch_set_active(mclbm_batch* b, const int32_t* active) {
  if (!b || !active) return fail(MCLBM_EINVAL, "NULL argument");
  for (int k = 0; k < b->n; ++k)
    if (active[k] && !b->active[k] && ((b->cav[k].t - b->t) & 1))
      return fail(MCLBM_EINVAL, "cavity " + std::to_string(k) + " cannot rejoin: step parity differs");
  for (int k = 0; k < b->n; ++k) b->active[k] = active[k] ? 1 : 0;
  return upload_tables(b);
}

int mclbm_batch_residual(mclbm_batch* b, double tol, double* out, int32_t* status) {
  if (!b || !out) return fail(MCLBM_EINVAL, "NULL argument");
  // every active cavity in three launches and one copy, then one synchronisation
  if (b->nr > 0) {
    const bool odd = (b->t & 1) != 0;
    int rc = dispatch_kinds(b->storage, b->idx32, b->nt, [&](auto k) {
      using S = typename decltype(k)::S;
      using I = typename decltype(k)::I;
      if (odd)
        k_residual_batch<true, S, I><<<b->nrt, 256, 0, b->stream>>>(b->d_desc(), b->d_red(), b->d_rtiles(), b->flip);
      else
        k_residual_batch<false, S, I><<<b->nrt, 256, 0, b->stream>>>(b->d_desc(), b->d_red(), b->d_rtiles(), b->flip);
      int r = launch_check("k_residual_batch");
      if (r) return r;
      k_sum_partials_batch<<<b->nr, 256, 0, b->stream>>>(b->d_red(), b->d_rlist(), b->d_rout());
      return launch_check("k_sum_partials_batch");
    });
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(b->h_red, b->d_rout(), (size_t)16 * b->nr * sizeof(double), hipMemcpyDeviceToHost,
                           b->stream));
  }
  HIP_TRY(hipStreamSynchronize(b->stream));
  for (int k = 0; k < b->n; ++k) {
    out[2 * k] = out[2 * k + 1] = NAN;
    if (status) status[k] = 3;
  }
  bool changed = false;
  for (int j = 0; j < b->nr; ++j) {
    const int k = b->host_rlist[j];
    double ru = 0.0, rt = 0.0;
    const int rc = finish_residual(b->h_red + 16 * j + 4, &ru, &rt);
    out[2 * k] = ru;
    out[2 * k + 1] = rt;
    const int32_t st = rc == MCLBM_EDIVERGED ? 2 : ((tol > 0.0 && ru < tol && rt < tol) ? 1 : 0);
    if (st != 0 && tol > 0.0) {
      b->active[k] = 0;
      changed = true;
    }
    if (status) status[k] = st;
  }
  g_err.clear();
  if (changed) return upload_tables(b);
  return MCLBM_OK;
}

int mclbm_batch_nusselt(mclbm_batch* b, double* out) {
  if (!b || !out) return fail(MCLBM_EINVAL, "NULL argument");
  // the active cavities in one launch and one copy; the inactive ones
  // (frozen, each at its own step parity) one by one, and only when their
  // state changed since their last reduction; one synchronisation
  if (b->nr > 0) {
    const bool odd = (b->t & 1) != 0;
    int rc = dispatch_kinds(b->storage, b->idx32, b->nt, [&](auto k) {
      using S = typename decltype(k)::S;
      using I = typename decltype(k)::I;
      if (odd)
        k_nusselt_batch<true, S, I><<<b->nr, 256, 0, b->stream>>>(b->d_desc(), b->d_red(), b->d_rlist(), b->flip,
                                                                  b->d_rout());
      else
        k_nusselt_batch<false, S, I><<<b->nr, 256, 0, b->stream>>>(b->d_desc(), b->d_red(), b->d_rlist(), b->flip,
                                                                   b->d_rout());
      return launch_check("k_nusselt_batch");
    });
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(b->h_red, b->d_rout(), (size_t)16 * b->nr * sizeof(double), hipMemcpyDeviceToHost,
                           b->stream));
  }
  if ((int)b->nu_t.size() != b->n) {
    b->nu_t.assign(b->n, -1);
    b->nu_epoch.assign(b->n, 0);
  }
  for (int k = 0; k < b->n; ++k)
    if (!b->active[k] && (b->nu_t[k] != b->cav[k].t || b->nu_epoch[k] != b->cav[k].epoch)) {
      const int rc = enqueue_nusselt(&b->cav[k], b->h_inactive(k));
      if (rc) {
        b->nu_t[k] = -1;
        return rc;
      }
      b->nu_t[k] = b->cav[k].t;
      b->nu_epoch[k] = b->cav[k].epoch;
    }
  HIP_TRY(hipStreamSynchronize(b->stream));
  for (int j = 0; j < b->nr; ++j) {
    const int k = b->host_rlist[j];
    (void)finish_nusselt(b->h_red + 16 * j, &out[3 * k], &out[3 * k + 1], &out[3 * k + 2]);
  }
  for (int k = 0; k < b->n; ++k)
    if (!b->active[k]) (void)finish_nusselt(b->h_inactive(k), &out[3 * k], &out[3 * k + 1], &out[3 * k + 2]);
  g_err.clear();
  return MCLBM_OK;
}

namespace {

void set_band2(mclbm_cavity* c, int band) {
  c->band2 = band;
  c->nblocks2 = (unsigned)c->strips2 * (unsigned)((c->cfg.ny + band - 1) / band);
}

void set_shape(mclbm_cavity* c, int si) {
  c->block = dim3(kShapes[si][0], kShapes[si][1], 1);
  c->tiles_x = (c->cfg.nx + kShapes[si][0] - 1) / kShapes[si][0];
}

}  // namespace

// Per size class (cavities of equal nx, ny), time each candidate with only
// that class active: the tile shape of the one-step kernel, or with two
// steps per launch the band height of the two-step tiles.
int mclbm_batch_autotune(mclbm_batch* b, int32_t steps) {
  if (!b) return fail(MCLBM_EINVAL, "batch is NULL");
  if (steps < 2) return fail(MCLBM_EINVAL, "autotune needs >= 2 steps per trial");
  HIP_TRY(hipStreamSynchronize(b->stream));
  const int saved_graph = b->graph_steps;
  b->graph_steps = 0;
  // size classes
  std::vector<std::pair<int, int>> classes;
  for (int k = 0; k < b->n; ++k) {
    auto key = std::make_pair(b->cav[k].cfg.nx, b->cav[k].cfg.ny);
    if (std::find(classes.begin(), classes.end(), key) == classes.end()) classes.push_back(key);
  }
  const int ncand = 4;
  auto apply = [&](mclbm_cavity* c, int ci) {
    if (b->two)
      set_band2(c, kBands2[ci]);
    else
      set_shape(c, ci);
  };
  auto trial_step = [&]() { return b->two ? batch_direct_step2(b) : batch_direct_step(b); };
  const int trials = b->two ? std::max(1, steps / 2) : steps;
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  int rc = MCLBM_OK;
  for (const auto& cl : classes) {
    float best = 1e30f;
    int best_c = 0;
    for (int ci = 0; ci < ncand && !rc; ++ci) {
      for (int k = 0; k < b->n; ++k) {
        mclbm_cavity* c = &b->cav[k];
        const bool in = c->cfg.nx == cl.first && c->cfg.ny == cl.second;
        b->active[k] = in ? 1 : 0;
        if (in) {
          apply(c, ci);
          rc = enqueue_init(c);
          if (rc) break;
        }
      }
      if (rc) break;
      b->t = 0;
      rc = upload_tables(b);
      if (rc) break;
      for (int w = 0; w < 2 && !rc; ++w) rc = trial_step();
      if (rc) break;
      HIP_TRY(hipEventRecord(e0, b->stream));
      for (int q = 0; q < trials && !rc; ++q) rc = trial_step();
      HIP_TRY(hipEventRecord(e1, b->stream));
      if (rc) break;
      hipError_t he = hipEventSynchronize(e1);
      if (he != hipSuccess) {
        rc = hip_fail(he, "hipEventSynchronize");
        break;
      }
      float ms = 0.0f;
      HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
      if (ms < best) {
        best = ms;
        best_c = ci;
      }
    }
    if (rc) break;
    for (int k = 0; k < b->n; ++k) {
      mclbm_cavity* c = &b->cav[k];
      if (c->cfg.nx == cl.first && c->cfg.ny == cl.second) apply(c, best_c);
    }
  }
  b->graph_steps = saved_graph;
  drop_graph(b);
  // then the schedule, every cavity active: the tiles (replayed from the
  // graph) or one workgroup per cavity
  if (!rc && percav_eligible(b)) {
    const bool prior = b->percav;
    rc = batch_reset_all(b);
    const int64_t n2 = std::max<int64_t>(std::max<int64_t>(2, steps & ~1), b->graph_steps);
    float ms[2] = {0.0f, 0.0f};
    for (int pc = 0; pc < 2 && !rc; ++pc) {
      b->percav = pc == 1;
      rc = mclbm_batch_step(b, n2);  // warm-up (and graph capture)
      if (rc) break;
      HIP_TRY(hipEventRecord(e0, b->stream));
      rc = mclbm_batch_step(b, n2);
      HIP_TRY(hipEventRecord(e1, b->stream));
      if (rc) break;
      hipError_t he = hipEventSynchronize(e1);
      if (he != hipSuccess) {
        rc = hip_fail(he, "hipEventSynchronize");
        break;
      }
      HIP_TRY(hipEventElapsedTime(&ms[pc], e0, e1));
    }
    b->percav = rc ? prior : ms[1] < ms[0];
    drop_graph(b);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  return batch_reset_all(b);
}

int mclbm_batch_tile_shape(const mclbm_batch* b, int32_t idx, int32_t* bx, int32_t* by) {
  if (!b || idx < 0 || idx >= b->n) return fail(MCLBM_EINVAL, "bad batch index");
  const mclbm_cavity& c = b->cav[idx];
  if (bx) *bx = b->two ? (int32_t)kStrip2 : (int32_t)c.block.x;
  if (by) *by = b->two ? (int32_t)c.band2 : (int32_t)c.block.y;
  return MCLBM_OK;
}

int mclbm_batch_reset(mclbm_batch* b) {
  if (!b) return fail(MCLBM_EINVAL, "batch is NULL");
  return batch_reset_all(b);
}

int32_t mclbm_batch_size(const mclbm_batch* b) { return b ? b->n : -1; }

int64_t mclbm_batch_time(const mclbm_batch* b, int32_t idx) {
  if (!b || idx < 0 || idx >= b->n) return -1;
  return b->cav[idx].t;
}

mclbm_cavity* mclbm_batch_cavity(mclbm_batch* b, int32_t idx) {
  if (!b || idx < 0 || idx >= b->n) return nullptr;
  return &b->cav[idx];
}

int mclbm_batch_destroy(mclbm_batch* b) {
  if (!b) return MCLBM_OK;
  hipError_t e = hipStreamSynchronize(b->stream);
  drop_graph(b);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  if (b->h_red) (void)hipHostFree(b->h_red);
  delete b;
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  return MCLBM_OK;
}

}  // extern "C"
