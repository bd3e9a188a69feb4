// HIP kernels and C ABI of the S2O4 DF-hybrid step for gfx950 (Zhang, Ji & Xu, arXiv:2402.10914).
//
// One step = [faces(stage 1)] [update 1] [faces(stage 2)] [update 2]:
//   faces:   one launch covers every x- and y-interface (of one grid, or of every grid of a batch).
//            A workgroup owns a tile of TF interfaces (along the normal) by TR interface segments
//            (along the tangential direction).  It stages the (TF+5) x (TR+4) cells and the alpha
//            halo in LDS once (ghost cells by index mapping), runs the normal reconstruction for
//            TR+4 segments per interface column into LDS, then the tangential reconstruction at
//            the two Gauss points of each of its TR segments, the flux and its time derivative, and
//            the DF of the Gauss points.  The thread that reconstructs a segment in the normal sweep
//            also owns it in the tangential sweep, so the normal derivatives stay in registers.
//   update:  one thread per cell assembles L and dL/dt from the four face sums (eqs. (3)-(4)) and
//            applies eq. (21); the second update also forms alpha^{n+1} (Section 3.2), checks
//            positivity and reduces the signal speed for the next dt (wavefront shuffle, LDS,
//            one 64-bit atomic max per workgroup on the bit pattern of a non-negative double).
// Every grid has its own control block (dt, time, status), so the grids of a batch advance with
// their own time steps; dt lives in device memory and the host never reads it inside a run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/dfweno.h"
#include "dfw_math.hpp"

namespace dfw {

// ------------------------------------------------------------------------------------------------
// Device-side descriptions.
// ------------------------------------------------------------------------------------------------
constexpr int kSpeedSlots = 64;  // one wavefront: the slots of a bank are reduced by one wave
struct Ctrl {
  // running max signal speed / dx for the next step (ping-pong banks).  Workgroup b adds its
  // maximum to slot b % kSpeedSlots of the bank, so that the atomics of a launch spread over
  // kSpeedSlots addresses instead of serialising on one; readers take the max over the slots.
  unsigned long long smax_bits[2][kSpeedSlots];
  double dt;                        // dt of the current step; 0 when the step is skipped (t_end reached)
  double t;                         // accumulated time (advanced by the last kernel of a step)
  int fail_at;                      // steps completed when a non-physical state was first met,
                                    // kNoFail if none; kernels of step n skip once fail_at <= n
  int pad[3];
};
constexpr int kNoFail = 0x7fffffff;

// Max over the slots of one bank (the bit patterns of non-negative doubles order as the values),
// taken by a whole wavefront: lane l reads slot l.  Every lane of the wave must be active.
__device__ __forceinline__ double bank_max(const Ctrl* ctrl, int bank) {
  double v = __longlong_as_double((long long)ctrl->smax_bits[bank][threadIdx.x & (kSpeedSlots - 1)]);
#pragma unroll
  for (int off = kSpeedSlots / 2; off > 0; off >>= 1) {
    const double o = __shfl_xor(v, off);
    v = o > v ? o : v;
  }
  return v;
}

// One grid: sizes, spacing, boundaries and element offsets of its arrays inside the (packed) state,
// alpha, stage and interface buffers.
struct GridDesc {
  int nx, ny, bc_x, bc_y;
  double dx, dy, inv_dx, inv_dy;
  long long w_off;   // W, W*, R: [4][ny][nx] at this offset
  long long a_off;   // alpha: [ny][nx]
  long long fx_off;  // x-interface data: [kFacePlanes][ny][nx+1]
  long long fy_off;  // y-interface data: [kFacePlanes][ny+1][nx]
};

struct Scheme {
  double gamma, cfl, dt_fixed, alpha_thres, eps, c1, c2, K;
  double d[4];
  // derived on the host (the same IEEE operations), so that kernels receive them as arguments instead
  // of computing them in vector registers, which they would hold for the whole launch
  double gm1, inv_gm1, dr[3], inv_d3, K2, k4K2;
  Coef<float> k32;  // every coefficient rounded to FP32 on the host, for the FP32 kernels
  int tl;  // non-linear time limiter (eqs. (27)-(29)) on
  int ts;  // time scheme: DFW_TIME_S2O4 (eq. (21)) or DFW_TIME_SSPRK3 (eq. (32))
  double t_end;  // > 0: stop at this time
  int sw;        // hybrid switch rule (0: max of the three DF values, eq. (42); 1: min; 2: own cell)
  int cw;        // 1: component-wise reconstruction of the conservative variables (ablation)
  int dfs;       // 1: alpha^{n+1} from the first stage's Gauss points instead of the last stage's
};

// OUT_OMEGA: time-limiter weight of each interface: with OUT_F (first stage) stored in plane 9, without
// (second stage) applied to the stored time derivative.
enum { OUT_F = 1, OUT_FT = 2, OUT_DF = 4, OUT_OMEGA = 8 };
constexpr int kFacePlanes = 10;  // F (4), dF/dt (4), DF product, time-limiter weight

// RULE >= 0 fixes the hybrid switch rule at compile time; RULE < 0 takes the rule of S.
template <class real, int RULE = -1>
__device__ __forceinline__ Coef<real> make_coef(const Scheme& S) {
  if constexpr (sizeof(real) == sizeof(float)) {
    Coef<real> k = S.k32;
    k.sw_rule = RULE >= 0 ? RULE : S.sw;
    return k;
  }
  Coef<real> k;
  k.gamma = real(S.gamma);
  k.gm1 = real(S.gm1);
  k.inv_gm1 = real(S.inv_gm1);
  k.alpha_thres = real(S.alpha_thres);
  k.eps = real(S.eps);
  k.c1 = real(S.c1);
  k.c2 = real(S.c2);
  k.K = real(S.K);
  for (int i = 0; i < 4; ++i) k.d[i] = real(S.d[i]);
  for (int i = 0; i < 3; ++i) k.dr[i] = real(S.dr[i]);
  k.inv_d3 = real(S.inv_d3);
  k.K2 = real(S.K2);
  k.k4K2 = real(S.k4K2);
  k.sw_rule = RULE >= 0 ? RULE : S.sw;
  return k;
}

// Workgroups are dispatched to the eight XCDs in turn (workgroup b to XCD b mod 8), and each XCD has
// its own L2.  Tile order for launches over interface tiles: the workgroups of one XCD take one
// contiguous run of the tile list, so neighbouring tiles, which stage overlapping halos, share an L2.
// A bijection of [0, n).
constexpr int kXcds = 8;
__host__ __device__ __forceinline__ int xcd_tile(int b, int n) {
  const int x = b % kXcds, k = b / kXcds, q = n / kXcds, r = n % kXcds;
  return x * q + (x < r ? x : r) + k;
}

// A value the same in every lane, moved to scalar registers (kernels at the register limit would
// otherwise hold values computed by vector instructions in vector registers).
__device__ __forceinline__ double uniform_value(double x) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(x);
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)b);
  const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ float uniform_value(float x) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}

__device__ __forceinline__ int bc_map(int i, int n, int bc) {
  if (bc == DFW_BC_PERIODIC) {
    int r = i % n;
    return r < 0 ? r + n : r;
  }
  return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

// ------------------------------------------------------------------------------------------------
// Interface kernel.
// Interface data: entries 0..3 = face-averaged flux (global components), 4..7 = its time
// derivative, 8 = product of the DF of the two Gauss points, 9 = time-limiter weight.
// Tile entry (batch form): x = grid, y = dir | (lead tile of its grid) << 1, z = f0, w = t0.
// ------------------------------------------------------------------------------------------------
template <int TF, int TR>
struct Tile {
  static constexpr int NR = TR + 4;   // segments incl. the normal-sweep halo
  static constexpr int NT = TF * NR;  // threads per workgroup
  static constexpr int WN = TF + 5;   // cells along the normal
  static constexpr int AN = TF + 3;   // alpha cells along the normal
};

template <int TF, int TR>
__host__ __device__ inline int tiles_x(int nx, int ny) { return ((nx + 1 + TF - 1) / TF) * ((ny + TR - 1) / TR); }

template <class real, int FLUX, int OUT, int TF, int TR>
__global__ __launch_bounds__(TF * (TR + 4)) void k_faces(const real* __restrict__ Wall, const real* __restrict__ Aall,
                                                         real* __restrict__ FXall, real* __restrict__ FYall,
                                                         Ctrl* __restrict__ ctrls, GridDesc G0,
                                                         const GridDesc* __restrict__ grids,
                                                         const int4* __restrict__ tiles, Scheme S, double dt_host,
                                                         int lead, int step, int nsteps, double* __restrict__ dt_hist) {
  using T = Tile<TF, TR>;
  __shared__ real sW[4][T::NR][T::WN];
  __shared__ real sA[T::NR][T::AN];
  __shared__ real sLine[8][T::NT];

  // ---- which grid and tile
  int gi = 0, dir, f0, t0;
  bool lead_tile;
  GridDesc G;
  if (tiles) {
    const int4 e = tiles[blockIdx.x];
    gi = e.x;
    dir = e.y & 1;
    lead_tile = (e.y >> 1) & 1;
    f0 = e.z;
    t0 = e.w;
    G = grids[gi];
  } else {
    G = G0;
    int b = xcd_tile(blockIdx.x, gridDim.x);
    const int nbx = tiles_x<TF, TR>(G.nx, G.ny);
    dir = b < nbx ? 0 : 1;
    if (dir) b -= nbx;
    const int ntf = dir ? (G.ny + 1 + TF - 1) / TF : (G.nx + 1 + TF - 1) / TF;
    f0 = (b % ntf) * TF;
    t0 = (b / ntf) * TR;
    lead_tile = blockIdx.x == 0;
  }
  const int nx = G.nx, ny = G.ny;
  const real* W = Wall + G.w_off;
  const real* alpha = Aall + G.a_off;
  real* FX = FXall + G.fx_off;
  real* FY = FYall + G.fy_off;
  const int Nn = dir ? ny : nx, Nt = dir ? nx : ny;
  const int bcn = dir ? G.bc_y : G.bc_x, bct = dir ? G.bc_x : G.bc_y;
  const real inv_dn = real(dir ? G.inv_dy : G.inv_dx), inv_dt = real(dir ? G.inv_dx : G.inv_dy);
  const size_t N = (size_t)nx * ny;
  const int tid = threadIdx.x;

  // ---- gather the tile's cells and alpha (ghost cells by index mapping) into registers, every load
  //      issued before the first is waited for, and before the control block is read, so that the
  //      tile's memory latency is paid once.  Component order local: 0 rho, 1 normal momentum,
  //      2 tangential momentum, 3 energy.  Tiles whose halo lies inside the grid (all but the tiles
  //      at the boundaries) skip the index map, whose periodic branch is an integer remainder per
  //      index; the test is uniform over the workgroup.  Threads past the end of the list reload the
  //      last entry (in bounds) and store nothing.
  constexpr int NWE = T::NR * T::WN, NAE = T::NR * T::AN;
  constexpr int IW = (NWE + T::NT - 1) / T::NT, IA = (NAE + T::NT - 1) / T::NT;
  const bool inner = f0 - 3 >= 0 && f0 + T::WN - 3 <= Nn && t0 - 2 >= 0 && t0 + T::NR - 2 <= Nt;
  auto map_n = [&](int i) { return inner ? i : bc_map(i, Nn, bcn); };
  auto map_t = [&](int i) { return inner ? i : bc_map(i, Nt, bct); };
  // LDS coordinates of list entry e over a patch of `width` cells along the normal: along the
  // normal fastest for x-interfaces (rows of the grid), along the tangent fastest for y-interfaces
  auto split = [&](int e, int width, int& nl, int& tl) {
    if (dir == 0) {
      tl = e / width;
      nl = e % width;
    } else {
      nl = e / T::NR;
      tl = e % T::NR;
    }
  };
  auto gcell = [&](int n, int t) -> size_t { return dir == 0 ? (size_t)t * nx + n : (size_t)n * nx + t; };
  real rw[IW][4], ra[IA];
#pragma unroll
  for (int it = 0; it < IW; ++it) {
    int nl, tl;
    split(min(tid + it * T::NT, NWE - 1), T::WN, nl, tl);
    const size_t g = gcell(map_n(f0 - 3 + nl), map_t(t0 - 2 + tl));
    rw[it][0] = W[g];
    rw[it][1] = W[(dir ? 2 : 1) * N + g];
    rw[it][2] = W[(dir ? 1 : 2) * N + g];
    rw[it][3] = W[3 * N + g];
  }
#pragma unroll
  for (int it = 0; it < IA; ++it) {
    int nl, tl;
    split(min(tid + it * T::NT, NAE - 1), T::AN, nl, tl);
    ra[it] = alpha[gcell(map_n(f0 - 2 + nl), map_t(t0 - 2 + tl))];
  }

  Ctrl* ctrl = ctrls + gi;
  if (ctrl->fail_at <= step) return;

  // ---- dt of this step.  The first launch of a step computes it (every tile the same value: t and
  // the speed slot do not change during this launch) and records it; later launches read it.  With
  // t_end > 0 the step that would pass t_end ends on it, and later steps are skipped (dt = 0).
  double dtd;
  if (lead) {
    dtd = dt_host > 0.0 ? dt_host : S.cfl / bank_max(ctrl, step & 1);
    if (S.t_end > 0.0) {
      const double rem = S.t_end - ctrl->t;
      if (dtd >= rem) dtd = rem > 0.0 ? rem : 0.0;
    }
  } else {
    dtd = dt_host > 0.0 ? dt_host : ctrl->dt;
  }
  if (lead && lead_tile) {
    if (dtd > 0.0 && tid < kSpeedSlots) ctrl->smax_bits[(step + 1) & 1][tid] = 0ull;
    if (tid == 0) {
      ctrl->dt = dtd;
      if (dt_hist) dt_hist[(size_t)gi * nsteps + step] = dtd;
    }
  }
  if (!(dtd > 0.0)) return;  // uniform over the launch
  const real dt = uniform_value(real(dtd));
  const Coef<real> k = make_coef<real>(S);

  // ---- the gathered tile into LDS
#pragma unroll
  for (int it = 0; it < IW; ++it) {
    const int e = tid + it * T::NT;
    if (e < NWE) {
      int nl, tl;
      split(e, T::WN, nl, tl);
#pragma unroll
      for (int c = 0; c < 4; ++c) sW[c][tl][nl] = rw[it][c];
    }
  }
#pragma unroll
  for (int it = 0; it < IA; ++it) {
    const int e = tid + it * T::NT;
    if (e < NAE) {
      int nl, tl;
      split(e, T::AN, nl, tl);
      sA[tl][nl] = ra[it];
    }
  }
  __syncthreads();

  // ---- item owned by this thread: interface column fl, segment row rr (row t = t0 - 2 + rr)
  int fl, rr;
  if (dir == 0) {
    fl = tid % TF;
    rr = tid / TF;
  } else {
    rr = tid % T::NR;
    fl = tid / T::NR;
  }
  const int rstride = dir == 0 ? TF : 1;  // thread-index distance between neighbouring rows
  const int f = f0 + fl, t = t0 - 2 + rr;
  const bool live1 = f <= Nn && t < Nt + 2;
  real wln[4] = {0, 0, 0, 0}, wrn[4] = {0, 0, 0, 0};
  real om = real(1);  // time-limiter weight of this interface segment, from the normal sweep
  real* const omp = (OUT & OUT_OMEGA) ? &om : nullptr;

  // ---- normal sweep (Section 3.1): line values of both sides and their normal derivatives
  if (live1) {
    real cell[6][4];
#pragma unroll
    for (int m = 0; m < 6; ++m)
#pragma unroll
      for (int c = 0; c < 4; ++c) cell[m][c] = sW[c][rr][fl + m];
    real wl[4], wr[4];
    if (S.cw)  // uniform over the launch
      normal_sweep<real, false>(cell, sA[rr][fl], sA[rr][fl + 1], sA[rr][fl + 2], sA[rr][fl + 3], inv_dn, k, wl, wr,
                                wln, wrn, omp);
    else
      normal_sweep<real, true>(cell, sA[rr][fl], sA[rr][fl + 1], sA[rr][fl + 2], sA[rr][fl + 3], inv_dn, k, wl, wr,
                               wln, wrn, omp);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      sLine[c][tid] = wl[c];
      sLine[4 + c][tid] = wr[c];
    }
  }
  __syncthreads();

  // ---- tangential sweep at the Gauss points, fluxes, DF
  const bool live2 = f <= Nn && rr >= 2 && rr < TR + 2 && t < Nt;
  if (!live2) return;
  real wa[4], wb[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    wa[c] = sW[c][rr][fl + 2];
    wb[c] = sW[c][rr][fl + 3];
  }
  real al[2][3];
#pragma unroll
  for (int side = 0; side < 2; ++side)  // DF of the cell on the same side as the Gauss point
#pragma unroll
    for (int q = 0; q < 3; ++q) al[side][q] = sA[rr - 1 + q][fl + 1 + side];
  auto line = [&](int side, int m, int c) -> real { return sLine[4 * side + c][tid + (m - 2) * rstride]; };
  real Fs[4], Fts[4], dfp;
  if (S.cw)
    segment_fluxes<real, FLUX, (OUT & OUT_F) != 0, (OUT & OUT_DF) != 0, false>(wa, wb, line, al, wln, wrn, dt, inv_dt,
                                                                               k, Fs, Fts, dfp);
  else
    segment_fluxes<real, FLUX, (OUT & OUT_F) != 0, (OUT & OUT_DF) != 0, true>(wa, wb, line, al, wln, wrn, dt, inv_dt,
                                                                              k, Fs, Fts, dfp);
  // ---- write face sums (quadrature weights 1/2), components back to the global order
  const size_t fstride = dir == 0 ? (size_t)ny * (nx + 1) : (size_t)(ny + 1) * nx;
  real* Fo = dir == 0 ? FX + (size_t)t * (nx + 1) + f : FY + (size_t)f * nx + t;
  const int cmap[4] = {0, dir ? 2 : 1, dir ? 1 : 2, 3};
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    if (OUT & OUT_F) Fo[cmap[c] * fstride] = real(0.5) * Fs[c];
    if (OUT & OUT_FT) {
      const real ft = real(0.5) * Fts[c];
      Fo[(4 + cmap[c]) * fstride] = ((OUT & OUT_OMEGA) && !(OUT & OUT_F)) ? om * ft : ft;
    }
  }
  if (OUT & OUT_DF) Fo[8 * fstride] = dfp;
  if ((OUT & OUT_OMEGA) && (OUT & OUT_F)) Fo[9 * fstride] = om;
}

// ------------------------------------------------------------------------------------------------
// Cell kernels: one thread per cell, 256 cells per workgroup, a workgroup never straddles grids.
// Cell-block entry (batch form): x = grid, y = first cell of the block.
// ------------------------------------------------------------------------------------------------
constexpr int kCellBlock = 256;

struct CellCtx {
  int gi;
  size_t o;  // cell index within its grid
  bool live;
  GridDesc G;
};

__device__ __forceinline__ CellCtx cell_ctx(const GridDesc& G0, const GridDesc* grids, const int2* cblocks) {
  CellCtx c;
  if (cblocks) {
    const int2 e = cblocks[blockIdx.x];
    c.gi = e.x;
    c.G = grids[e.x];
    c.o = (size_t)e.y + threadIdx.x;
  } else {
    c.gi = 0;
    c.G = G0;
    c.o = (size_t)blockIdx.x * kCellBlock + threadIdx.x;
  }
  c.live = c.o < (size_t)c.G.nx * c.G.ny;
  return c;
}

template <class real>
__device__ __forceinline__ void face_sum(const real* FX, const real* FY, const GridDesc& G, int i, int j, int base,
                                         real* out) {
  // no contraction here: the x and y contributions are rounded alike, so a transposed grid
  // (x <-> y, U <-> V) gives a bitwise transposed result
#pragma clang fp contract(off)
  const int nx = G.nx, ny = G.ny;
  const size_t sx = (size_t)ny * (nx + 1), sy = (size_t)(ny + 1) * nx;
  const size_t w = (size_t)j * (nx + 1) + i, s = (size_t)j * nx + i;
  const real ix = real(G.inv_dx), iy = real(G.inv_dy);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const real* fx = FX + (base + c) * sx;
    const real* fy = FY + (base + c) * sy;
    real ax = (fx[w] - fx[w + 1]) * ix;
    real ay = (fy[s] - fy[s + nx]) * iy;
    out[c] = ax + ay;
  }
}

// The time derivative of eq. (28): each face's dL/dt weighted by its time-limiter weight (plane 9).
template <class real>
__device__ __forceinline__ void face_sum_limited(const real* FX, const real* FY, const GridDesc& G, int i, int j,
                                                 real* out) {
#pragma clang fp contract(off)
  const int nx = G.nx, ny = G.ny;
  const size_t sx = (size_t)ny * (nx + 1), sy = (size_t)(ny + 1) * nx;
  const size_t w = (size_t)j * (nx + 1) + i, s = (size_t)j * nx + i;
  const real ix = real(G.inv_dx), iy = real(G.inv_dy);
  const real* ox = FX + 9 * sx;
  const real* oy = FY + 9 * sy;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const real* fx = FX + (4 + c) * sx;
    const real* fy = FY + (4 + c) * sy;
    real ax = (ox[w] * fx[w] - ox[w + 1] * fx[w + 1]) * ix;
    real ay = (oy[s] * fy[s] - oy[s + nx] * fy[s + nx]) * iy;
    out[c] = ax + ay;
  }
}

template <class real>
__global__ __launch_bounds__(kCellBlock) void k_update1(const real* __restrict__ Wall, const real* __restrict__ FXall,
                                                        const real* __restrict__ FYall, real* __restrict__ Wsall,
                                                        real* __restrict__ Rall, Ctrl* __restrict__ ctrls, GridDesc G0,
                                                        const GridDesc* __restrict__ grids,
                                                        const int2* __restrict__ cblocks, int step, int tl) {
  const CellCtx C = cell_ctx(G0, grids, cblocks);
  Ctrl* ctrl = ctrls + C.gi;
  if (ctrl->fail_at <= step || !(ctrl->dt > 0.0) || !C.live) return;
  const GridDesc& G = C.G;
  const size_t N = (size_t)G.nx * G.ny, o = C.o;
  const int i = (int)(o % G.nx), j = (int)(o / G.nx);
  const real* W = Wall + G.w_off;
  real* Ws = Wsall + G.w_off;
  real* R = Rall + G.w_off;
  const real dt = real(ctrl->dt);
  real L[4], Lt[4];
  face_sum(FXall + G.fx_off, FYall + G.fy_off, G, i, j, 0, L);
  face_sum(FXall + G.fx_off, FYall + G.fy_off, G, i, j, 4, Lt);
  const real h1 = real(0.5) * dt, h2 = dt * dt * real(0.125), r2 = dt * dt * real(1.0 / 6.0);
  if (tl) {  // eq. (27): R = W + dt L + dt^2/2 L_t - dt^2/3 ~L_t (W* as without the limiter)
    real Ltl[4];
    face_sum_limited(FXall + G.fx_off, FYall + G.fy_off, G, i, j, Ltl);
    const real q2 = dt * dt * real(0.5), q3 = dt * dt * real(1.0 / 3.0);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      real w = W[c * N + o];
      Ws[c * N + o] = w + h1 * L[c] + h2 * Lt[c];
      R[c * N + o] = w + dt * L[c] + q2 * Lt[c] - q3 * Ltl[c];
    }
    return;
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    real w = W[c * N + o];
    Ws[c * N + o] = w + h1 * L[c] + h2 * Lt[c];
    R[c * N + o] = w + dt * L[c] + r2 * Lt[c];
  }
}

template <class real>
__device__ __forceinline__ bool cell_speed(const real* w, const Scheme& S, const GridDesc& G, double& s) {
  const real g = real(S.gamma);
  real ir = real(1) / w[0];
  real u = w[1] * ir, v = w[2] * ir;
  real p = real(S.gamma - 1.0) * (w[3] - real(0.5) * (w[1] * u + w[2] * v));
  bool ok = w[0] > real(0) && p > real(0) && isfinite(w[1]) && isfinite(w[2]) && isfinite(w[3]) && isfinite(p);
  real c = sqrt(g * p * ir);
  real sx = (fabs(u) + c) * real(G.inv_dx), sy = (fabs(v) + c) * real(G.inv_dy);
  s = ok ? double(sx > sy ? sx : sy) : 0.0;
  return ok;
}

// Workgroup max of a non-negative double and OR of a flag, then one atomic each (the max into the
// workgroup's slot of the bank).  A flag records step_done as the failing step; it stops the
// kernels of later steps only, so every workgroup of the launch that finds it still writes its
// cells and the stored state does not depend on the order in which workgroups run.
__device__ __forceinline__ void block_reduce_commit(double s, int bad, Ctrl* ctrl, int slot, int step_done) {
  __shared__ double red[kCellBlock / 64];
  __shared__ int redb[kCellBlock / 64];
  for (int off = 32; off > 0; off >>= 1) {
    double o = __shfl_xor(s, off);
    s = o > s ? o : s;
    bad |= __shfl_xor(bad, off);
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  if (lane == 0) {
    red[wv] = s;
    redb[wv] = bad;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < nw; ++q) {
      s = red[q] > s ? red[q] : s;
      bad |= redb[q];
    }
    if (s > 0.0)
      atomicMax(&ctrl->smax_bits[slot][blockIdx.x & (kSpeedSlots - 1)], (unsigned long long)__double_as_longlong(s));
    if (bad) atomicMin(&ctrl->fail_at, step_done);
  }
}

// Stores the new state w of cell (i, j), its alpha^{n+1} (product of the DF of its four faces,
// Section 3.2) and returns whether the state is physical, with its signal speed in s.
template <class real>
__device__ __forceinline__ int finish_cell(const real* w, real* W, real* Aall, const real* FX, const real* FY,
                                           const GridDesc& G, const Scheme& S, size_t o, int i, int j, double& s) {
  const size_t N = (size_t)G.nx * G.ny;
#pragma unroll
  for (int c = 0; c < 4; ++c) W[c * N + o] = w[c];
  const int nx = G.nx, ny = G.ny;
  const size_t sx = (size_t)ny * (nx + 1), sy = (size_t)(ny + 1) * nx;
  const size_t fw = (size_t)j * (nx + 1) + i;
  const real* ax = FX + 8 * sx;
  const real* ay = FY + 8 * sy;
  Aall[G.a_off + o] = (ax[fw] * ax[fw + 1]) * (ay[o] * ay[o + nx]);
  return cell_speed(w, S, G, s) ? 0 : 1;
}

// The last kernel of a step advances the grid's time, from the thread of its cell 0 (no other
// thread of the launch reads t); the step that reaches t_end ends exactly on it.
__device__ __forceinline__ void advance_time(Ctrl* ctrl, const Scheme& S, double dtd) {
  const double t = ctrl->t;
  ctrl->t = (S.t_end > 0.0 && dtd >= S.t_end - t) ? S.t_end : t + dtd;
}

template <class real>
__global__ __launch_bounds__(kCellBlock) void k_update2(real* __restrict__ Wall, real* __restrict__ Aall,
                                                        const real* __restrict__ Rall, const real* __restrict__ FXall,
                                                        const real* __restrict__ FYall, Ctrl* __restrict__ ctrls,
                                                        GridDesc G0, const GridDesc* __restrict__ grids,
                                                        const int2* __restrict__ cblocks, Scheme S, int step) {
  const CellCtx C = cell_ctx(G0, grids, cblocks);
  Ctrl* ctrl = ctrls + C.gi;
  const double dtd = ctrl->dt;
  if (ctrl->fail_at <= step || !(dtd > 0.0)) return;  // uniform over the workgroup: one grid per workgroup
  const GridDesc& G = C.G;
  double s = 0.0;
  int bad = 0;
  if (C.live) {
    const size_t N = (size_t)G.nx * G.ny, o = C.o;
    const int i = (int)(o % G.nx), j = (int)(o / G.nx);
    const real* FX = FXall + G.fx_off;
    const real* FY = FYall + G.fy_off;
    const real* R = Rall + G.w_off;
    const real dt = real(dtd);
    if (o == 0) advance_time(ctrl, S, dtd);
    real Lt[4], w[4];
    face_sum(FX, FY, G, i, j, 4, Lt);
    const real r3 = dt * dt * real(1.0 / 3.0);
#pragma unroll
    for (int c = 0; c < 4; ++c) w[c] = R[c * N + o] + r3 * Lt[c];
    bad = finish_cell(w, Wall + G.w_off, Aall, FX, FY, G, S, o, i, j, s);
  }
  block_reduce_commit(s, bad, ctrl, (step + 1) & 1, step + 1);
}

// Eq. (32), SSP-RK3, first two stages, from the face fluxes of the stage state:
//   STAGE 1: U = W^n + dt L(W^n);   STAGE 2: U = 3/4 W^n + 1/4 W1 + 1/4 dt L(W1).
template <class real, int STAGE>
__global__ __launch_bounds__(kCellBlock) void k_rk_stage(const real* __restrict__ Wall, const real* __restrict__ W1all,
                                                         const real* __restrict__ FXall, const real* __restrict__ FYall,
                                                         real* __restrict__ Uall, Ctrl* __restrict__ ctrls, GridDesc G0,
                                                         const GridDesc* __restrict__ grids,
                                                         const int2* __restrict__ cblocks, int step) {
  const CellCtx C = cell_ctx(G0, grids, cblocks);
  Ctrl* ctrl = ctrls + C.gi;
  if (ctrl->fail_at <= step || !(ctrl->dt > 0.0) || !C.live) return;
  const GridDesc& G = C.G;
  const size_t N = (size_t)G.nx * G.ny, o = C.o;
  const int i = (int)(o % G.nx), j = (int)(o / G.nx);
  const real* W = Wall + G.w_off;
  real* U = Uall + G.w_off;
  const real dt = real(ctrl->dt);
  real L[4];
  face_sum(FXall + G.fx_off, FYall + G.fy_off, G, i, j, 0, L);
  if (STAGE == 1) {
#pragma unroll
    for (int c = 0; c < 4; ++c) U[c * N + o] = W[c * N + o] + dt * L[c];
  } else {
    const real* W1 = W1all + G.w_off;
    const real q = real(0.25) * dt;
#pragma unroll
    for (int c = 0; c < 4; ++c) U[c * N + o] = (real(0.75) * W[c * N + o] + real(0.25) * W1[c * N + o]) + q * L[c];
  }
}

// Eq. (32), third stage: W^{n+1} = 1/3 W^n + 2/3 W2 + 2/3 dt L(W2), with alpha^{n+1} from this stage's
// Gauss points and the CFL reduction of the new state (as the second S2O4 stage).
template <class real>
__global__ __launch_bounds__(kCellBlock) void k_rk_final(real* __restrict__ Wall, real* __restrict__ Aall,
                                                         const real* __restrict__ W2all, const real* __restrict__ FXall,
                                                         const real* __restrict__ FYall, Ctrl* __restrict__ ctrls,
                                                         GridDesc G0, const GridDesc* __restrict__ grids,
                                                         const int2* __restrict__ cblocks, Scheme S, int step) {
  const CellCtx C = cell_ctx(G0, grids, cblocks);
  Ctrl* ctrl = ctrls + C.gi;
  const double dtd = ctrl->dt;
  if (ctrl->fail_at <= step || !(dtd > 0.0)) return;
  const GridDesc& G = C.G;
  double s = 0.0;
  int bad = 0;
  if (C.live) {
    const size_t N = (size_t)G.nx * G.ny, o = C.o;
    const int i = (int)(o % G.nx), j = (int)(o / G.nx);
    const real* FX = FXall + G.fx_off;
    const real* FY = FYall + G.fy_off;
    const real* W = Wall + G.w_off;
    const real* W2 = W2all + G.w_off;
    const real dt = real(dtd);
    if (o == 0) advance_time(ctrl, S, dtd);
    real L[4], w[4];
    face_sum(FX, FY, G, i, j, 0, L);
    const real a = real(1.0 / 3.0), b = real(2.0 / 3.0), q = real(2.0 / 3.0) * dt;
#pragma unroll
    for (int c = 0; c < 4; ++c) w[c] = (a * W[c * N + o] + b * W2[c * N + o]) + q * L[c];
    bad = finish_cell(w, Wall + G.w_off, Aall, FX, FY, G, S, o, i, j, s);
  }
  block_reduce_commit(s, bad, ctrl, (step + 1) & 1, step + 1);
}

template <class real>
__global__ __launch_bounds__(kCellBlock) void k_speed(const real* __restrict__ Wall, Ctrl* __restrict__ ctrls,
                                                      GridDesc G0, const GridDesc* __restrict__ grids,
                                                      const int2* __restrict__ cblocks, Scheme S, int slot) {
  const CellCtx C = cell_ctx(G0, grids, cblocks);
  Ctrl* ctrl = ctrls + C.gi;
  const GridDesc& G = C.G;
  double s = 0.0;
  int bad = 0;
  if (C.live) {
    const size_t N = (size_t)G.nx * G.ny, o = C.o;
    const real* W = Wall + G.w_off;
    real w[4] = {W[o], W[N + o], W[2 * N + o], W[3 * N + o]};
    bad = cell_speed(w, S, G, s) ? 0 : 1;
  }
  block_reduce_commit(s, bad, ctrl, slot, 0);
}

__global__ void k_ctrl_init(Ctrl* ctrls, int n) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  Ctrl* c = ctrls + g;
  for (int q = 0; q < kSpeedSlots; ++q) c->smax_bits[0][q] = c->smax_bits[1][q] = 0ull;
  c->dt = 0.0;
  c->t = 0.0;
  c->fail_at = kNoFail;
}

template <class real>
__global__ __launch_bounds__(kCellBlock) void k_assemble(const real* __restrict__ FX, const real* __restrict__ FY,
                                                         real* __restrict__ L, real* __restrict__ Lt,
                                                         real* __restrict__ an, GridDesc G) {
  const size_t N = (size_t)G.nx * G.ny, o = (size_t)blockIdx.x * kCellBlock + threadIdx.x;
  if (o >= N) return;
  const int i = (int)(o % G.nx), j = (int)(o / G.nx);
  real a[4], b[4];
  face_sum(FX, FY, G, i, j, 0, a);
  face_sum(FX, FY, G, i, j, 4, b);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    L[c * N + o] = a[c];
    Lt[c * N + o] = b[c];
  }
  if (an) {
    const int nx = G.nx, ny = G.ny;
    const size_t sx = (size_t)ny * (nx + 1), sy = (size_t)(ny + 1) * nx;
    const size_t fw = (size_t)j * (nx + 1) + i;
    an[o] = (FX[8 * sx + fw] * FX[8 * sx + fw + 1]) * (FY[8 * sy + o] * FY[8 * sy + o + nx]);
  }
}

// ------------------------------------------------------------------------------------------------
// Host side.
// ------------------------------------------------------------------------------------------------
static thread_local std::string g_err;

static dfw_status fail(dfw_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Event-based per-kernel timing for benchmarks (see dfw_profile).
struct Profiler {
  bool on = false;
  struct Rec {
    int kind;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  hipEvent_t take() {
    if (used == pool.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      pool.push_back(e);
    }
    return pool[used++];
  }
};
static Profiler g_prof;

template <class Launch>
static void timed(int kind, hipStream_t st, Launch launch) {
  if (!g_prof.on) {
    launch();
    return;
  }
  hipEvent_t a = g_prof.take(), b = g_prof.take();
  const bool ok_a = a && hipEventRecord(a, st) == hipSuccess;
  launch();
  const bool ok_b = b && hipEventRecord(b, st) == hipSuccess;
  if (ok_a && ok_b) g_prof.recs.push_back({kind, a, b});  // a launch without both events is not timed
}

// Interface tile shapes (TF interfaces x TR segments); index 0 is the library default.
struct TileShape {
  int tf, tr;
};
static const TileShape kShapes[] = {{8, 28}, {16, 28}, {8, 60}, {16, 12}, {4, 60}};
constexpr int kNumShapes = sizeof(kShapes) / sizeof(kShapes[0]);

static int shape_tiles(int shape, int nx, int ny) {
  const TileShape s = kShapes[shape];
  return ((nx + 1 + s.tf - 1) / s.tf) * ((ny + s.tr - 1) / s.tr) + ((ny + 1 + s.tf - 1) / s.tf) * ((nx + s.tr - 1) / s.tr);
}

struct FaceLaunch {
  int shape, flux, out;
  int nblocks;
  const int4* tiles;
  const GridDesc* grids;
  GridDesc G0;
  Ctrl* ctrls;
  Scheme S;
  double dt_host;
  int lead, step, nsteps;
  double* dt_hist;
};

template <class real, int FLUX, int OUT, int TF, int TR>
static void launch_faces_t(const FaceLaunch& L, const real* W, const real* A, real* FX, real* FY, hipStream_t st) {
  hipLaunchKernelGGL((k_faces<real, FLUX, OUT, TF, TR>), dim3(L.nblocks), dim3(TF * (TR + 4)), 0, st, W, A, FX, FY,
                     L.ctrls, L.G0, L.grids, L.tiles, L.S, L.dt_host, L.lead, L.step, L.nsteps, L.dt_hist);
}

template <class real, int FLUX, int OUT>
static void launch_faces_shape(const FaceLaunch& L, const real* W, const real* A, real* FX, real* FY, hipStream_t st) {
  switch (L.shape) {
    case 1: launch_faces_t<real, FLUX, OUT, 16, 28>(L, W, A, FX, FY, st); break;
    case 2: launch_faces_t<real, FLUX, OUT, 8, 60>(L, W, A, FX, FY, st); break;
    case 3: launch_faces_t<real, FLUX, OUT, 16, 12>(L, W, A, FX, FY, st); break;
    case 4: launch_faces_t<real, FLUX, OUT, 4, 60>(L, W, A, FX, FY, st); break;
    default: launch_faces_t<real, FLUX, OUT, 8, 28>(L, W, A, FX, FY, st); break;
  }
}

template <class real, int OUT>
static void launch_faces_out(const FaceLaunch& L, const real* W, const real* A, real* FX, real* FY, hipStream_t st) {
  if (L.flux == DFW_FLUX_LF) launch_faces_shape<real, DFW_FLUX_LF, OUT>(L, W, A, FX, FY, st);
  else launch_faces_shape<real, DFW_FLUX_GKS, OUT>(L, W, A, FX, FY, st);
}

template <class real>
static void launch_faces(const FaceLaunch& L, const real* W, const real* A, real* FX, real* FY, hipStream_t st) {
  // fluxes without time derivatives: the SSP-RK3 stages, which run with the LF flux only
  if (L.out == OUT_F) launch_faces_shape<real, DFW_FLUX_LF, OUT_F>(L, W, A, FX, FY, st);
  else if (L.out == (OUT_F | OUT_DF)) launch_faces_shape<real, DFW_FLUX_LF, OUT_F | OUT_DF>(L, W, A, FX, FY, st);
  else if (L.out == (OUT_F | OUT_FT)) launch_faces_out<real, OUT_F | OUT_FT>(L, W, A, FX, FY, st);
  // the DF taken from the first stage (df_stage = 1): the second stage writes no DF
  else if (L.out == OUT_FT) launch_faces_out<real, OUT_FT>(L, W, A, FX, FY, st);
  else if (L.out == (OUT_FT | OUT_OMEGA)) launch_faces_out<real, OUT_FT | OUT_OMEGA>(L, W, A, FX, FY, st);
  else if (L.out == (OUT_F | OUT_FT | OUT_DF | OUT_OMEGA))
    launch_faces_out<real, OUT_F | OUT_FT | OUT_DF | OUT_OMEGA>(L, W, A, FX, FY, st);
  else if (L.out == (OUT_FT | OUT_DF)) launch_faces_out<real, OUT_FT | OUT_DF>(L, W, A, FX, FY, st);
  else if (L.out == (OUT_F | OUT_FT | OUT_OMEGA)) launch_faces_out<real, OUT_F | OUT_FT | OUT_OMEGA>(L, W, A, FX, FY, st);
  else if (L.out == (OUT_FT | OUT_DF | OUT_OMEGA))
    launch_faces_out<real, OUT_FT | OUT_DF | OUT_OMEGA>(L, W, A, FX, FY, st);
  else launch_faces_out<real, OUT_F | OUT_FT | OUT_DF>(L, W, A, FX, FY, st);
}

// Workspace of a single grid.
struct WsLayout {
  size_t ws_off, r_off, fx_off, fy_off, ctrl_off, total;
};

static WsLayout layout(const dfw_grid* g, size_t es) {
  WsLayout L;
  size_t N = (size_t)g->nx * g->ny;
  size_t off = 0;
  L.ws_off = off;
  off = align256(off + 4 * N * es);
  L.r_off = off;
  off = align256(off + 4 * N * es);
  L.fx_off = off;
  off = align256(off + kFacePlanes * (size_t)g->ny * (g->nx + 1) * es);
  L.fy_off = off;
  off = align256(off + kFacePlanes * (size_t)(g->ny + 1) * g->nx * es);
  L.ctrl_off = off;
  off = align256(off + sizeof(Ctrl));
  L.total = off;
  return L;
}

static dfw_status check_grid(const dfw_grid* g) {
  if (!g) return fail(DFW_EINVAL, "null grid");
  if (g->nx < 1 || g->ny < 1) return fail(DFW_EINVAL, "nx and ny must be >= 1");
  if ((size_t)g->nx * g->ny > ((size_t)1 << 31)) return fail(DFW_EINVAL, "grid too large (nx*ny > 2^31)");
  if (!(g->dx > 0) || !(g->dy > 0)) return fail(DFW_EINVAL, "dx and dy must be > 0");
  if ((g->bc_x != DFW_BC_PERIODIC && g->bc_x != DFW_BC_TRANSMISSIVE) ||
      (g->bc_y != DFW_BC_PERIODIC && g->bc_y != DFW_BC_TRANSMISSIVE))
    return fail(DFW_EINVAL, "unknown boundary condition");
  return DFW_OK;
}

static dfw_status check_params(const dfw_params* p, int32_t dtype) {
  if (!p) return fail(DFW_EINVAL, "null params");
  if (!(p->gamma > 1.0)) return fail(DFW_EINVAL, "gamma must be > 1");
  if (p->flux != DFW_FLUX_LF && p->flux != DFW_FLUX_GKS) return fail(DFW_EINVAL, "unknown flux");
  if (!(p->d_h > 0 && p->d_h < 1) || !(p->d_l >= 0 && p->d_l <= 1)) return fail(DFW_EINVAL, "d_h in (0,1), d_l in [0,1]");
  if (!(p->eps_weno > 0)) return fail(DFW_EINVAL, "eps_weno must be > 0");
  if (!(p->c1 >= 0) || !(p->c2 >= 0)) return fail(DFW_EINVAL, "c1, c2 must be >= 0");
  if (p->tile < 0 || p->tile >= kNumShapes) return fail(DFW_EINVAL, "tile must be in [0, dfw_num_tiles())");
  if (p->time_limiter != 0 && p->time_limiter != 1) return fail(DFW_EINVAL, "time_limiter must be 0 or 1");
  if (p->time_scheme != DFW_TIME_S2O4 && p->time_scheme != DFW_TIME_SSPRK3)
    return fail(DFW_EINVAL, "time_scheme must be DFW_TIME_S2O4 or DFW_TIME_SSPRK3");
  if (p->time_scheme == DFW_TIME_SSPRK3 && (p->flux != DFW_FLUX_LF || p->time_limiter))
    return fail(DFW_EINVAL, "SSP-RK3 runs with the LF flux and without the time limiter");
  if (!(p->t_end >= 0.0)) return fail(DFW_EINVAL, "t_end must be >= 0 (0: no end time)");
  if (p->switch_rule < 0 || p->switch_rule > 2) return fail(DFW_EINVAL, "switch_rule must be 0, 1 or 2");
  if (p->componentwise != 0 && p->componentwise != 1) return fail(DFW_EINVAL, "componentwise must be 0 or 1");
  if (p->df_stage != 0 && p->df_stage != 1) return fail(DFW_EINVAL, "df_stage must be 0 or 1");
  if (dtype != DFW_F64 && dtype != DFW_F32) return fail(DFW_EDTYPE, "dtype must be DFW_F64 or DFW_F32");
  return DFW_OK;
}

static dfw_status check_common(const dfw_grid* g, const dfw_params* p, int32_t dtype) {
  dfw_status s = check_grid(g);
  return s != DFW_OK ? s : check_params(p, dtype);
}

static Scheme make_scheme(const dfw_params* p) {
  Scheme S;
  S.gamma = p->gamma;
  S.cfl = p->cfl;
  S.dt_fixed = p->dt_fixed;
  S.alpha_thres = p->alpha_thres;
  S.eps = p->eps_weno;
  S.c1 = p->c1;
  S.c2 = p->c2;
  S.K = (4.0 - 2.0 * p->gamma) / (p->gamma - 1.0);
  S.d[3] = p->d_h;
  S.d[0] = (1.0 - p->d_h) * (1.0 - p->d_l) / 2.0;
  S.d[1] = (1.0 - p->d_h) * p->d_l;
  S.d[2] = S.d[0];
  S.gm1 = S.gamma - 1.0;
  S.inv_gm1 = 1.0 / (S.gamma - 1.0);
  for (int i = 0; i < 3; ++i) S.dr[i] = S.d[i] / S.d[3];
  S.inv_d3 = 1.0 / S.d[3];
  S.K2 = S.K + 2.0;
  S.k4K2 = 4.0 / (S.K + 2.0);
  Coef<float>& f = S.k32;  // round to nearest, as a conversion on the device
  f.gamma = float(S.gamma);
  f.gm1 = float(S.gm1);
  f.inv_gm1 = float(S.inv_gm1);
  f.alpha_thres = float(S.alpha_thres);
  f.eps = float(S.eps);
  f.c1 = float(S.c1);
  f.c2 = float(S.c2);
  f.K = float(S.K);
  for (int i = 0; i < 4; ++i) f.d[i] = float(S.d[i]);
  for (int i = 0; i < 3; ++i) f.dr[i] = float(S.dr[i]);
  f.inv_d3 = float(S.inv_d3);
  f.K2 = float(S.K2);
  f.k4K2 = float(S.k4K2);
  f.sw_rule = p->switch_rule;
  S.tl = p->time_limiter;
  S.ts = p->time_scheme;
  S.t_end = p->t_end;
  S.sw = p->switch_rule;
  S.cw = p->componentwise;
  S.dfs = p->df_stage;
  return S;
}

static GridDesc make_desc(const dfw_grid* g) {
  GridDesc G;
  G.nx = g->nx;
  G.ny = g->ny;
  G.bc_x = g->bc_x;
  G.bc_y = g->bc_y;
  G.dx = g->dx;
  G.dy = g->dy;
  G.inv_dx = 1.0 / g->dx;
  G.inv_dy = 1.0 / g->dy;
  G.w_off = G.a_off = G.fx_off = G.fy_off = 0;
  return G;
}

#define HIP_TRY(x)                                                                               \
  do {                                                                                           \
    hipError_t e_ = (x);                                                                         \
    if (e_ != hipSuccess) return fail(DFW_EHIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

static unsigned cell_blocks(const GridDesc& G) { return (unsigned)(((size_t)G.nx * G.ny + kCellBlock - 1) / kCellBlock); }

// The kernels of nsteps time steps (S2O4, or SSP-RK3) on `st` (no synchronisation).  Single grid: grids/tiles/cblocks
// are null and G0 describes the grid; batch: the tables describe every grid.
struct NoHook {
  void operator()(int) const {}
};

// before_step(n) is called on the host before the kernels of step n are enqueued.
template <class real, class Hook = NoHook>
static void enqueue_steps(real* W, real* A, real* Ws, real* R, real* FX, real* FY, Ctrl* ctrls, int nctrl,
                          const GridDesc& G0, const GridDesc* grids, const int4* tiles, int ntiles,
                          const int2* cblocks, int ncblocks, const dfw_params* p, int nsteps, double* dt_hist,
                          hipStream_t st, Hook before_step = Hook()) {
  const Scheme S = make_scheme(p);
  FaceLaunch L;
  L.shape = p->tile;
  L.flux = p->flux;
  L.nblocks = ntiles;
  L.tiles = tiles;
  L.grids = grids;
  L.G0 = G0;
  L.ctrls = ctrls;
  L.S = S;
  const double dt_first = p->dt_fixed > 0 ? p->dt_fixed : 0.0;  // later launches of a step read ctrl->dt
  L.nsteps = nsteps;
  const unsigned nb = (unsigned)ncblocks;
  hipLaunchKernelGGL(k_ctrl_init, dim3((nctrl + 63) / 64), dim3(64), 0, st, ctrls, nctrl);
  timed(DFW_K_SPEED, st, [&] {
    hipLaunchKernelGGL(k_speed<real>, dim3(nb), dim3(kCellBlock), 0, st, W, ctrls, G0, grids, cblocks, S, 0);
  });
  if (S.ts == DFW_TIME_SSPRK3) {
    for (int n = 0; n < nsteps; ++n) {
      before_step(n);
      L.step = n;
      L.out = OUT_F | (S.dfs ? OUT_DF : 0);
      L.lead = 1;
      L.dt_host = dt_first;
      L.dt_hist = dt_hist;
      timed(DFW_K_RK_FACES, st, [&] { launch_faces<real>(L, W, A, FX, FY, st); });
      timed(DFW_K_RK_UPDATE, st, [&] {
        hipLaunchKernelGGL((k_rk_stage<real, 1>), dim3(nb), dim3(kCellBlock), 0, st, W, (const real*)nullptr, FX, FY,
                           Ws, ctrls, G0, grids, cblocks, n);
      });
      L.out = OUT_F;
      L.lead = 0;
      L.dt_host = 0.0;
      L.dt_hist = nullptr;
      timed(DFW_K_RK_FACES, st, [&] { launch_faces<real>(L, Ws, A, FX, FY, st); });
      timed(DFW_K_RK_UPDATE, st, [&] {
        hipLaunchKernelGGL((k_rk_stage<real, 2>), dim3(nb), dim3(kCellBlock), 0, st, W, Ws, FX, FY, R, ctrls, G0,
                           grids, cblocks, n);
      });
      L.out = OUT_F | (S.dfs ? 0 : OUT_DF);
      timed(DFW_K_RK_FACES, st, [&] { launch_faces<real>(L, R, A, FX, FY, st); });
      timed(DFW_K_RK_UPDATE, st, [&] {
        hipLaunchKernelGGL(k_rk_final<real>, dim3(nb), dim3(kCellBlock), 0, st, W, A, R, FX, FY, ctrls, G0, grids,
                           cblocks, S, n);
      });
    }
    return;
  }
  for (int n = 0; n < nsteps; ++n) {
    before_step(n);
    L.step = n;
    L.out = OUT_F | OUT_FT | (S.tl ? OUT_OMEGA : 0) | (S.dfs ? OUT_DF : 0);
    L.lead = 1;
    L.dt_host = dt_first;
    L.dt_hist = dt_hist;
    timed(DFW_K_FACES1, st, [&] { launch_faces<real>(L, W, A, FX, FY, st); });
    timed(DFW_K_UPDATE1, st, [&] {
      hipLaunchKernelGGL(k_update1<real>, dim3(nb), dim3(kCellBlock), 0, st, W, FX, FY, Ws, R, ctrls, G0, grids,
                         cblocks, n, S.tl);
    });
    L.out = OUT_FT | (S.dfs ? 0 : OUT_DF) | (S.tl ? OUT_OMEGA : 0);
    L.lead = 0;
    L.dt_host = 0.0;
    L.dt_hist = nullptr;
    timed(DFW_K_FACES2, st, [&] { launch_faces<real>(L, Ws, A, FX, FY, st); });
    timed(DFW_K_UPDATE2, st, [&] {
      hipLaunchKernelGGL(k_update2<real>, dim3(nb), dim3(kCellBlock), 0, st, W, A, R, FX, FY, ctrls, G0, grids,
                         cblocks, S, n);
    });
  }
}

template <class real>
static dfw_status run_impl(real* W, real* A, const dfw_grid* g, const dfw_params* p, int nsteps, char* ws,
                           double* dt_hist, double* t_out, int32_t* fail_step, hipStream_t st) {
  WsLayout L = layout(g, sizeof(real));
  Ctrl* ctrl = (Ctrl*)(ws + L.ctrl_off);
  const GridDesc G = make_desc(g);
  enqueue_steps<real>(W, A, (real*)(ws + L.ws_off), (real*)(ws + L.r_off), (real*)(ws + L.fx_off),
                      (real*)(ws + L.fy_off), ctrl, 1, G, nullptr, nullptr, shape_tiles(p->tile, g->nx, g->ny),
                      nullptr, (int)cell_blocks(G), p, nsteps, dt_hist, st);
  HIP_TRY(hipGetLastError());
  Ctrl h;
  HIP_TRY(hipMemcpyAsync(&h, ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (t_out) *t_out = h.t;
  if (fail_step) *fail_step = h.fail_at != kNoFail ? h.fail_at : -1;
  if (h.fail_at != kNoFail)
    return fail(DFW_ENONPHYS, "non-physical state after " + std::to_string(h.fail_at) + " steps");
  return DFW_OK;
}

}  // namespace dfw

#include "dfw_reverse.hpp"

// ================================================================================================
// Batched ragged grids.
// ================================================================================================
struct dfw_batch {
  int ngrids = 0;
  int32_t dtype = DFW_F64;
  dfw_params params{};
  std::vector<dfw::GridDesc> grids;
  std::vector<int4> tiles;
  std::vector<int2> cblocks;
  size_t w_elems = 0, a_elems = 0, fx_elems = 0, fy_elems = 0;
  size_t ws_off = 0, r_off = 0, fx_off = 0, fy_off = 0, ctrl_off = 0, ws_bytes = 0;
  void* dtab = nullptr;  // device copy of grids | tiles | cblocks (owned by the plan)
  dfw::GridDesc* d_grids = nullptr;
  int4* d_tiles = nullptr;
  int2* d_cblocks = nullptr;
  // captured rollout
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  hipStream_t cap_stream = nullptr;
  void *g_W = nullptr, *g_A = nullptr, *g_ws = nullptr, *g_dth = nullptr;
  int g_nsteps = -1;
};

namespace dfw {

static void build_tiles(dfw_batch* b, int order) {
  const TileShape s = kShapes[b->params.tile];
  std::vector<int> idx(b->ngrids);
  for (int g = 0; g < b->ngrids; ++g) idx[g] = g;
  if (order == DFW_ORDER_LARGEST_FIRST)
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int c) {
      return (long long)b->grids[a].nx * b->grids[a].ny > (long long)b->grids[c].nx * b->grids[c].ny;
    });
  b->tiles.clear();
  std::vector<std::vector<int4>> per_grid(b->ngrids);
  for (int g : idx) {
    const GridDesc& G = b->grids[g];
    bool first = true;
    for (int dir = 0; dir < 2; ++dir) {
      const int Nn = dir ? G.ny : G.nx, Nt = dir ? G.nx : G.ny;
      for (int t0 = 0; t0 < Nt; t0 += s.tr)
        for (int f0 = 0; f0 <= Nn; f0 += s.tf) {
          per_grid[g].push_back(make_int4(g, dir | (first ? 2 : 0), f0, t0));
          first = false;
        }
    }
  }
  std::vector<int4> list;
  if (order == DFW_ORDER_INTERLEAVED) {  // round-robin over grids: neighbouring workgroups differ in grid
    size_t longest = 0;
    for (int g : idx) longest = std::max(longest, per_grid[g].size());
    for (size_t k = 0; k < longest; ++k)
      for (int g : idx)
        if (k < per_grid[g].size()) list.push_back(per_grid[g][k]);
  } else {
    for (int g : idx) list.insert(list.end(), per_grid[g].begin(), per_grid[g].end());
  }
  // workgroup b runs list entry xcd_tile(b): each XCD takes a contiguous run of the order above
  const int n = (int)list.size();
  b->tiles.resize(list.size());
  for (int w = 0; w < n; ++w) b->tiles[w] = list[xcd_tile(w, n)];
}

template <class real>
static void batch_enqueue(dfw_batch* b, void* W, void* A, char* ws, int nsteps, double* dth, hipStream_t st) {
  enqueue_steps<real>((real*)W, (real*)A, (real*)(ws + b->ws_off), (real*)(ws + b->r_off), (real*)(ws + b->fx_off),
                      (real*)(ws + b->fy_off), (Ctrl*)(ws + b->ctrl_off), b->ngrids, b->grids[0], b->d_grids,
                      b->d_tiles, (int)b->tiles.size(), b->d_cblocks, (int)b->cblocks.size(), &b->params, nsteps, dth,
                      st);
}

static void drop_graph(dfw_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

}  // namespace dfw

using namespace dfw;

extern "C" {

size_t dfw_workspace_bytes(const dfw_grid* grid, int32_t dtype) {
  if (!grid || grid->nx < 1 || grid->ny < 1) return 0;
  return layout(grid, dtype == DFW_F32 ? 4 : 8).total;
}

static dfw_status check_ws(const dfw_grid* g, int32_t dtype, void* ws, size_t ws_bytes) {
  if (!ws) return fail(DFW_EWORKSPACE, "workspace is null");
  if (((uintptr_t)ws) & 255) return fail(DFW_EWORKSPACE, "workspace must be 256-byte aligned");
  size_t need = layout(g, dtype == DFW_F32 ? 4 : 8).total;
  if (ws_bytes < need) return fail(DFW_EWORKSPACE, "workspace too small: need " + std::to_string(need) + " bytes");
  return DFW_OK;
}

static dfw_status check_run(void* W, void* alpha, const dfw_grid* grid, const dfw_params* params, int32_t nsteps,
                            int32_t dtype) {
  dfw_status s = check_common(grid, params, dtype);
  if (s != DFW_OK) return s;
  if (!W || !alpha) return fail(DFW_EINVAL, "W and alpha must be non-null");
  if (nsteps < 0) return fail(DFW_EINVAL, "nsteps must be >= 0");
  if (!(params->dt_fixed > 0) && !(params->cfl > 0)) return fail(DFW_EINVAL, "need cfl > 0 or dt_fixed > 0");
  return DFW_OK;
}

dfw_status dfw_run(void* W, void* alpha, const dfw_grid* grid, const dfw_params* params, int32_t nsteps,
                   int32_t dtype, void* ws, size_t ws_bytes, double* dt_hist_dev, double* t_out,
                   int32_t* fail_step, void* stream) {
  dfw_status s = check_run(W, alpha, grid, params, nsteps, dtype);
  if (s != DFW_OK) return s;
  if ((s = check_ws(grid, dtype, ws, ws_bytes)) != DFW_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  if (dtype == DFW_F64)
    return run_impl<double>((double*)W, (double*)alpha, grid, params, nsteps, (char*)ws, dt_hist_dev, t_out,
                            fail_step, st);
  return run_impl<float>((float*)W, (float*)alpha, grid, params, nsteps, (char*)ws, dt_hist_dev, t_out, fail_step,
                         st);
}

}  // extern "C"

// ---- workspace in a fixed device array (dfw_run_noalloc) ----
// Each GPU the library runs on holds its own copy of `scratch` until the process ends.  On the host
// the name stands for a host-side shadow, not a device address: kernels and copies take the
// address hipGetSymbolAddress returns for the current device, looked up once per device.
static __device__ __align__(256) unsigned char scratch[DFW_NOALLOC_SCRATCH_BYTES];

namespace dfw {
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

static dfw_status scratch_for_current_device(char** out) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(DFW_EHIP, "device index " + std::to_string(dev) + " out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(DFW_EHIP, std::string("hipGetSymbolAddress of the scratch array: ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = (char*)g_scratch_ptr[dev];
  return DFW_OK;
}
}  // namespace dfw

extern "C" {

dfw_status dfw_run_noalloc(void* W, void* alpha, const dfw_grid* grid, const dfw_params* params, int32_t nsteps,
                           int32_t dtype, double* dt_hist_dev, double* t_out, int32_t* fail_step, void* stream) {
  dfw_status s = check_run(W, alpha, grid, params, nsteps, dtype);
  if (s != DFW_OK) return s;
  const size_t need = layout(grid, dtype == DFW_F32 ? 4 : 8).total;
  if (need > (size_t)DFW_NOALLOC_SCRATCH_BYTES)
    return fail(DFW_EWORKSPACE, "grid " + std::to_string(grid->nx) + "x" + std::to_string(grid->ny) + " needs " +
                                    std::to_string(need) + " bytes of workspace; the fixed scratch array holds " +
                                    std::to_string((size_t)DFW_NOALLOC_SCRATCH_BYTES) + " (use dfw_run)");
  char* ws = nullptr;
  if ((s = scratch_for_current_device(&ws)) != DFW_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  if (dtype == DFW_F64)
    return run_impl<double>((double*)W, (double*)alpha, grid, params, nsteps, ws, dt_hist_dev, t_out, fail_step, st);
  return run_impl<float>((float*)W, (float*)alpha, grid, params, nsteps, ws, dt_hist_dev, t_out, fail_step, st);
}

dfw_status dfw_max_speed(const void* W, const dfw_grid* grid, const dfw_params* params, int32_t dtype, void* ws,
                         size_t ws_bytes, double* smax, int32_t* nonphys, void* stream) {
  dfw_status s = check_common(grid, params, dtype);
  if (s != DFW_OK) return s;
  if (!W) return fail(DFW_EINVAL, "W must be non-null");
  if ((s = check_ws(grid, dtype, ws, ws_bytes)) != DFW_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  WsLayout L = layout(grid, dtype == DFW_F32 ? 4 : 8);
  Ctrl* ctrl = (Ctrl*)((char*)ws + L.ctrl_off);
  const GridDesc G = make_desc(grid);
  const Scheme S = make_scheme(params);
  hipLaunchKernelGGL(k_ctrl_init, dim3(1), dim3(64), 0, st, ctrl, 1);
  if (dtype == DFW_F64)
    hipLaunchKernelGGL(k_speed<double>, dim3(cell_blocks(G)), dim3(kCellBlock), 0, st, (const double*)W, ctrl, G,
                       nullptr, nullptr, S, 0);
  else
    hipLaunchKernelGGL(k_speed<float>, dim3(cell_blocks(G)), dim3(kCellBlock), 0, st, (const float*)W, ctrl, G,
                       nullptr, nullptr, S, 0);
  HIP_TRY(hipGetLastError());
  Ctrl h;
  HIP_TRY(hipMemcpyAsync(&h, ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  unsigned long long bits = 0ull;
  for (int q = 0; q < kSpeedSlots; ++q) bits = h.smax_bits[0][q] > bits ? h.smax_bits[0][q] : bits;
  double v;
  std::memcpy(&v, &bits, sizeof(double));
  if (smax) *smax = v;
  if (nonphys) *nonphys = h.fail_at != kNoFail ? 1 : 0;
  return DFW_OK;
}

dfw_status dfw_rhs(const void* W, const void* alpha, const dfw_grid* grid, const dfw_params* params, int32_t dtype,
                   double dt, void* L, void* Lt, void* alpha_new, void* ws, size_t ws_bytes, void* stream) {
  dfw_status s = check_common(grid, params, dtype);
  if (s != DFW_OK) return s;
  if (!W || !alpha || !L || !Lt) return fail(DFW_EINVAL, "W, alpha, L and Lt must be non-null");
  if (!(dt > 0)) return fail(DFW_EINVAL, "dt must be > 0");
  if ((s = check_ws(grid, dtype, ws, ws_bytes)) != DFW_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  WsLayout Lw = layout(grid, dtype == DFW_F32 ? 4 : 8);
  Ctrl* ctrl = (Ctrl*)((char*)ws + Lw.ctrl_off);
  const GridDesc G = make_desc(grid);
  FaceLaunch FL;
  FL.shape = params->tile;
  FL.flux = params->flux;
  FL.out = OUT_F | OUT_FT | OUT_DF;
  FL.nblocks = shape_tiles(params->tile, grid->nx, grid->ny);
  FL.tiles = nullptr;
  FL.grids = nullptr;
  FL.G0 = G;
  FL.ctrls = ctrl;
  FL.S = make_scheme(params);
  FL.dt_host = dt;
  FL.lead = 0;
  FL.step = 0;
  FL.nsteps = 1;
  FL.dt_hist = nullptr;
  hipLaunchKernelGGL(k_ctrl_init, dim3(1), dim3(64), 0, st, ctrl, 1);
  if (dtype == DFW_F64) {
    double* FX = (double*)((char*)ws + Lw.fx_off);
    double* FY = (double*)((char*)ws + Lw.fy_off);
    launch_faces<double>(FL, (const double*)W, (const double*)alpha, FX, FY, st);
    hipLaunchKernelGGL(k_assemble<double>, dim3(cell_blocks(G)), dim3(kCellBlock), 0, st, FX, FY, (double*)L,
                       (double*)Lt, (double*)alpha_new, G);
  } else {
    float* FX = (float*)((char*)ws + Lw.fx_off);
    float* FY = (float*)((char*)ws + Lw.fy_off);
    launch_faces<float>(FL, (const float*)W, (const float*)alpha, FX, FY, st);
    hipLaunchKernelGGL(k_assemble<float>, dim3(cell_blocks(G)), dim3(kCellBlock), 0, st, FX, FY, (float*)L,
                       (float*)Lt, (float*)alpha_new, G);
  }
  HIP_TRY(hipGetLastError());
  return DFW_OK;
}

// ---- batched ragged grids ----

dfw_status dfw_batch_plan(const dfw_grid* grids, int32_t ngrids, const dfw_params* params, int32_t dtype,
                          int32_t order, dfw_batch** out) {
  if (!out) return fail(DFW_EINVAL, "out is null");
  *out = nullptr;
  if (!grids || ngrids < 1) return fail(DFW_EINVAL, "need at least one grid");
  dfw_status s = check_params(params, dtype);
  if (s != DFW_OK) return s;
  if (!(params->dt_fixed > 0) && !(params->cfl > 0)) return fail(DFW_EINVAL, "need cfl > 0 or dt_fixed > 0");
  if (order < 0 || order > DFW_ORDER_INTERLEAVED) return fail(DFW_EINVAL, "unknown sweep order");
  dfw_batch* b = new dfw_batch();
  b->ngrids = ngrids;
  b->dtype = dtype;
  b->params = *params;
  const size_t es = dtype == DFW_F32 ? 4 : 8;
  for (int g = 0; g < ngrids; ++g) {
    if ((s = check_grid(&grids[g])) != DFW_OK) {
      delete b;
      return fail(s, "grid " + std::to_string(g) + ": " + g_err);
    }
    GridDesc G = make_desc(&grids[g]);
    const size_t N = (size_t)G.nx * G.ny;
    G.w_off = (long long)b->w_elems;
    G.a_off = (long long)b->a_elems;
    G.fx_off = (long long)b->fx_elems;
    G.fy_off = (long long)b->fy_elems;
    b->w_elems += 4 * N;
    b->a_elems += N;
    b->fx_elems += kFacePlanes * (size_t)G.ny * (G.nx + 1);
    b->fy_elems += kFacePlanes * (size_t)(G.ny + 1) * G.nx;
    b->grids.push_back(G);
    const size_t ncb = (N + kCellBlock - 1) / kCellBlock;
    for (size_t k = 0; k < ncb; ++k) b->cblocks.push_back(make_int2(g, (int)(k * kCellBlock)));
  }
  if (b->w_elems >= ((size_t)1 << 40)) {
    delete b;
    return fail(DFW_EINVAL, "batch too large (more than 2^38 cells)");
  }
  build_tiles(b, order);
  // one launch covers every tile (cell block) of the batch: the work items of a launch must stay below
  // 2^32, and the block counts are passed to the launch as int
  const size_t max_items = 0xffffffffull;
  const size_t tile_threads = (size_t)kShapes[b->params.tile].tf * (kShapes[b->params.tile].tr + 4);
  if (b->tiles.size() > (size_t)INT32_MAX || b->cblocks.size() > (size_t)INT32_MAX ||
      b->tiles.size() * tile_threads > max_items || b->cblocks.size() * kCellBlock > max_items) {
    const size_t nt = b->tiles.size(), nc = b->cblocks.size();
    delete b;
    return fail(DFW_EINVAL, "batch too large for one launch: " + std::to_string(nt) + " interface tiles, " +
                                std::to_string(nc) + " cell blocks");
  }
  size_t off = 0;
  b->ws_off = off;
  off = align256(off + b->w_elems * es);
  b->r_off = off;
  off = align256(off + b->w_elems * es);
  b->fx_off = off;
  off = align256(off + b->fx_elems * es);
  b->fy_off = off;
  off = align256(off + b->fy_elems * es);
  b->ctrl_off = off;
  off = align256(off + (size_t)ngrids * sizeof(Ctrl));
  b->ws_bytes = off;
  const size_t tb_g = align256(b->grids.size() * sizeof(GridDesc));
  const size_t tb_t = align256(b->tiles.size() * sizeof(int4));
  const size_t tb_c = align256(b->cblocks.size() * sizeof(int2));
  hipError_t e = hipMalloc(&b->dtab, tb_g + tb_t + tb_c);
  if (e != hipSuccess) {
    delete b;
    return fail(DFW_EHIP, std::string("hipMalloc of the batch tables: ") + hipGetErrorString(e));
  }
  b->d_grids = (GridDesc*)b->dtab;
  b->d_tiles = (int4*)((char*)b->dtab + tb_g);
  b->d_cblocks = (int2*)((char*)b->dtab + tb_g + tb_t);
  if (hipMemcpy(b->d_grids, b->grids.data(), b->grids.size() * sizeof(GridDesc), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b->d_tiles, b->tiles.data(), b->tiles.size() * sizeof(int4), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b->d_cblocks, b->cblocks.data(), b->cblocks.size() * sizeof(int2), hipMemcpyHostToDevice) !=
          hipSuccess) {
    (void)hipFree(b->dtab);
    delete b;
    return fail(DFW_EHIP, "copying the batch tables failed");
  }
  *out = b;
  return DFW_OK;
}

dfw_status dfw_batch_layout(const dfw_batch* b, int64_t* w_offsets, int64_t* a_offsets, size_t* w_elems,
                            size_t* a_elems, size_t* ws_bytes) {
  if (!b) return fail(DFW_EINVAL, "null batch");
  for (int g = 0; g < b->ngrids; ++g) {
    if (w_offsets) w_offsets[g] = b->grids[g].w_off;
    if (a_offsets) a_offsets[g] = b->grids[g].a_off;
  }
  if (w_elems) *w_elems = b->w_elems;
  if (a_elems) *a_elems = b->a_elems;
  if (ws_bytes) *ws_bytes = b->ws_bytes;
  return DFW_OK;
}

dfw_status dfw_batch_run(dfw_batch* b, void* W_flat, void* alpha_flat, int32_t nsteps, void* ws, size_t ws_bytes,
                         int32_t use_graph, double* dt_hist_dev, double* t_out, int32_t* fail_steps, void* stream) {
  if (!b) return fail(DFW_EINVAL, "null batch");
  if (!W_flat || !alpha_flat) return fail(DFW_EINVAL, "W_flat and alpha_flat must be non-null");
  if (nsteps < 0) return fail(DFW_EINVAL, "nsteps must be >= 0");
  if (!ws) return fail(DFW_EWORKSPACE, "workspace is null");
  if (((uintptr_t)ws) & 255) return fail(DFW_EWORKSPACE, "workspace must be 256-byte aligned");
  if (ws_bytes < b->ws_bytes) return fail(DFW_EWORKSPACE, "workspace too small: need " + std::to_string(b->ws_bytes));
  hipStream_t st = (hipStream_t)stream;
  if (use_graph) {
    const bool same = b->exec && b->g_W == W_flat && b->g_A == alpha_flat && b->g_ws == ws &&
                      b->g_dth == (void*)dt_hist_dev && b->g_nsteps == nsteps;
    if (!same) {
      drop_graph(b);
      if (!b->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
      HIP_TRY(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
      const bool prof = g_prof.on;
      g_prof.on = false;  // no events inside the graph
      if (b->dtype == DFW_F64) batch_enqueue<double>(b, W_flat, alpha_flat, (char*)ws, nsteps, dt_hist_dev, b->cap_stream);
      else batch_enqueue<float>(b, W_flat, alpha_flat, (char*)ws, nsteps, dt_hist_dev, b->cap_stream);
      g_prof.on = prof;
      hipError_t le = hipGetLastError();
      hipError_t ce = hipStreamEndCapture(b->cap_stream, &b->graph);
      if (le != hipSuccess || ce != hipSuccess) {
        drop_graph(b);
        return fail(DFW_EHIP, std::string("graph capture failed: ") + hipGetErrorString(le != hipSuccess ? le : ce));
      }
      HIP_TRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
      b->g_W = W_flat;
      b->g_A = alpha_flat;
      b->g_ws = ws;
      b->g_dth = (void*)dt_hist_dev;
      b->g_nsteps = nsteps;
    }
    hipError_t ge = hipSuccess;
    timed(DFW_K_GRAPH, st, [&] { ge = hipGraphLaunch(b->exec, st); });
    HIP_TRY(ge);
  } else {
    if (b->dtype == DFW_F64) batch_enqueue<double>(b, W_flat, alpha_flat, (char*)ws, nsteps, dt_hist_dev, st);
    else batch_enqueue<float>(b, W_flat, alpha_flat, (char*)ws, nsteps, dt_hist_dev, st);
  }
  HIP_TRY(hipGetLastError());
  std::vector<Ctrl> h(b->ngrids);
  HIP_TRY(hipMemcpyAsync(h.data(), (char*)ws + b->ctrl_off, b->ngrids * sizeof(Ctrl), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  int nbad = 0;
  for (int g = 0; g < b->ngrids; ++g) {
    if (t_out) t_out[g] = h[g].t;
    if (fail_steps) fail_steps[g] = h[g].fail_at != kNoFail ? h[g].fail_at : -1;
    nbad += h[g].fail_at != kNoFail ? 1 : 0;
  }
  if (nbad) return fail(DFW_ENONPHYS, std::to_string(nbad) + " grid(s) met a non-physical state");
  return DFW_OK;
}

void dfw_batch_free(dfw_batch* b) {
  if (!b) return;
  drop_graph(b);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  if (b->dtab) (void)hipFree(b->dtab);
  delete b;
}

// ---- reverse mode ----

size_t dfw_checkpoint_bytes(const dfw_grid* grid, int32_t dtype, int32_t nsteps, int32_t ckpt_every) {
  if (!grid || grid->nx < 1 || grid->ny < 1 || nsteps < 0 || ckpt_every < 1) return 0;
  return ckpt_layout(grid, dtype == DFW_F32 ? 4 : 8, nsteps, ckpt_every).total;
}

static dfw_status check_ckpt(const dfw_grid* g, int32_t dtype, int32_t nsteps, int32_t every, const void* ckpt,
                             size_t ckpt_bytes) {
  if (every < 1) return fail(DFW_EINVAL, "ckpt_every must be >= 1");
  if (nsteps < 0) return fail(DFW_EINVAL, "nsteps must be >= 0");
  const size_t need = ckpt_layout(g, dtype == DFW_F32 ? 4 : 8, nsteps, every).total;
  if (need && !ckpt) return fail(DFW_EINVAL, "checkpoint store is null");
  if (((uintptr_t)ckpt) & 255) return fail(DFW_EINVAL, "checkpoint store must be 256-byte aligned");
  if (ckpt_bytes < need) return fail(DFW_EINVAL, "checkpoint store too small: need " + std::to_string(need) + " bytes");
  return DFW_OK;
}

dfw_status dfw_run_ckpt(void* W, void* alpha, const dfw_grid* grid, const dfw_params* params, int32_t nsteps,
                        int32_t dtype, int32_t ckpt_every, void* ckpt, size_t ckpt_bytes, void* ws,
                        size_t ws_bytes, double* dt_hist_dev, double* t_out, int32_t* fail_step, void* stream) {
  dfw_status s = check_common(grid, params, dtype);
  if (s != DFW_OK) return s;
  if (!W || !alpha) return fail(DFW_EINVAL, "W and alpha must be non-null");
  if (!dt_hist_dev && nsteps > 0) return fail(DFW_EINVAL, "dt_hist_dev is required");
  if (!(params->dt_fixed > 0) && !(params->cfl > 0)) return fail(DFW_EINVAL, "need cfl > 0 or dt_fixed > 0");
  if ((s = check_ckpt(grid, dtype, nsteps, ckpt_every, ckpt, ckpt_bytes)) != DFW_OK) return s;
  if ((s = check_ws(grid, dtype, ws, ws_bytes)) != DFW_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  if (dtype == DFW_F64)
    return run_ckpt_impl<double>((double*)W, (double*)alpha, grid, params, nsteps, ckpt_every, (char*)ckpt, (char*)ws,
                                 dt_hist_dev, t_out, fail_step, st);
  return run_ckpt_impl<float>((float*)W, (float*)alpha, grid, params, nsteps, ckpt_every, (char*)ckpt, (char*)ws,
                              dt_hist_dev, t_out, fail_step, st);
}

size_t dfw_adjoint_workspace_bytes(const dfw_grid* grid, int32_t dtype, int32_t ckpt_every) {
  if (!grid || grid->nx < 1 || grid->ny < 1 || ckpt_every < 1) return 0;
  return adj_layout(grid, dtype == DFW_F32 ? 4 : 8, ckpt_every).total;
}

dfw_status dfw_adjoint(const dfw_grid* grid, const dfw_params* params, int32_t dtype, int32_t nsteps,
                       int32_t ckpt_every, const void* ckpt, size_t ckpt_bytes, const double* dt_hist_dev,
                       const void* gW_final, const void* gA_final, void* gW0, void* gA0, void* ws, size_t ws_bytes,
                       void* stream) {
  dfw_status s = check_common(grid, params, dtype);
  if (s != DFW_OK) return s;
  if (dtype != DFW_F64) return fail(DFW_EDTYPE, "the adjoint is implemented in FP64 only");
  if (params->time_limiter) return fail(DFW_EINVAL, "the adjoint does not cover the time limiter");
  if (params->time_scheme != DFW_TIME_S2O4) return fail(DFW_EINVAL, "the adjoint covers the S2O4 step only");
  if (params->t_end > 0.0) return fail(DFW_EINVAL, "the adjoint takes its time steps from dt_hist; t_end must be 0");
  if (params->componentwise || params->df_stage)
    return fail(DFW_EINVAL, "the adjoint covers the characteristic reconstruction and the DF of the last stage");
  if (!gW_final || !gW0) return fail(DFW_EINVAL, "gW_final and gW0 must be non-null");
  if (!dt_hist_dev && nsteps > 0) return fail(DFW_EINVAL, "dt_hist_dev is required");
  if ((s = check_ckpt(grid, dtype, nsteps, ckpt_every, ckpt, ckpt_bytes)) != DFW_OK) return s;
  if (!ws) return fail(DFW_EWORKSPACE, "workspace is null");
  if (((uintptr_t)ws) & 255) return fail(DFW_EWORKSPACE, "workspace must be 256-byte aligned");
  const size_t need = adj_layout(grid, 8, ckpt_every).total;
  if (ws_bytes < need) return fail(DFW_EWORKSPACE, "workspace too small: need " + std::to_string(need) + " bytes");
  hipStream_t st = (hipStream_t)stream;
  if (params->flux == DFW_FLUX_LF)
    return adjoint_impl<double, DFW_FLUX_LF>(grid, params, nsteps, ckpt_every, (const char*)ckpt, dt_hist_dev,
                                             (const double*)gW_final, (const double*)gA_final, (double*)gW0,
                                             (double*)gA0, (char*)ws, st);
  return adjoint_impl<double, DFW_FLUX_GKS>(grid, params, nsteps, ckpt_every, (const char*)ckpt, dt_hist_dev,
                                            (const double*)gW_final, (const double*)gA_final, (double*)gW0,
                                            (double*)gA0, (char*)ws, st);
}

// ---- measurement ----

dfw_status dfw_profile(int32_t enable) {
  g_prof.recs.clear();
  g_prof.used = 0;
  g_prof.on = enable != 0;
  return DFW_OK;
}

dfw_status dfw_profile_read(double* ms, int64_t* launches, int32_t n) {
  if (!ms || !launches || n < 0) return fail(DFW_EINVAL, "null output arrays");
  for (int k = 0; k < n; ++k) {
    ms[k] = 0.0;
    launches[k] = 0;
  }
  for (const auto& r : g_prof.recs) {
    HIP_TRY(hipEventSynchronize(r.b));
    float e = 0.f;
    HIP_TRY(hipEventElapsedTime(&e, r.a, r.b));
    if (r.kind >= 0 && r.kind < n) {
      ms[r.kind] += e;
      launches[r.kind] += 1;
    }
  }
  return DFW_OK;
}

int32_t dfw_num_tiles(void) { return kNumShapes; }

dfw_status dfw_tile_shape(int32_t tile, int32_t* tf, int32_t* tr) {
  if (tile < 0 || tile >= kNumShapes) return fail(DFW_EINVAL, "tile out of range");
  if (tf) *tf = kShapes[tile].tf;
  if (tr) *tr = kShapes[tile].tr;
  return DFW_OK;
}

const char* dfw_last_error(void) { return g_err.c_str(); }

}  // extern "C"
