// Reverse mode of the S2O4 step (adjoint kernels and their orchestration with step checkpointing).
// Compiled inside dfw_step.hip, so it shares the forward kernels, the workspace helpers and the
// error and profiling state of the library.
//
// The adjoint of one stage operator (U, alpha) -> (L, dL/dt, alpha_new), for given adjoints of its
// outputs, takes two kernels:
//   k_adj_faces   one workgroup per interface tile (the forward tiling; x and y interfaces in one
//                 launch).  It stages the cells and alpha with a 4-row tangential halo in LDS, and
//                 the seed terms of the cells beside its interfaces (formed once per cell),
//                 recomputes the normal-sweep line values of TR+8 rows, runs the segment adjoint
//                 (Gauss-point reconstruction, flux, DF) of TR+4 segment rows, sums for each row the
//                 line adjoints of the five segments that read it (five LDS rounds in a fixed order),
//                 runs the normal-sweep adjoint of the rows the tile owns, and writes per row the
//                 adjoints of the seven cells its two interfaces' normal stencils cover and of the
//                 three DFs they read, the two interfaces' terms summed in the tile: 31 values, each
//                 with exactly one writer (no atomics).
//   k_adj_gather  one thread per cell: sums the window-buffer entries of the cell (ghost cells fold
//                 back through the boundary map) in a fixed order, and applies the stage recurrences
//                 of eq. (21) in reverse.
// Results are bitwise reproducible.
#pragma once

#include "dfw_adjoint.hpp"

namespace dfw {

constexpr int kAdjSlots = 31;  // per tile row: 7 stencil cells x 4 components, then 3 DF values

template <int TF, int TR>
struct AdjTile {
  static constexpr int NR = TR + 4;   // segment rows of the tile
  static constexpr int NP = TF * NR;  // interface segments = lane pairs
  static constexpr int NT = 2 * NP;   // threads: one per segment side
  static constexpr int NQ = TR + 8;   // normal-sweep rows
  static constexpr int WN = TF + 5;   // cells along the normal
  static constexpr int AN = TF + 3;   // alpha cells along the normal
};

// Value of lane (lane ^ X) within the lane's quad, X = 1, 2, 3, as two DPP quad permutes of the
// 32-bit halves (vector moves, instead of a permute through the LDS unit).  Every lane of the quad
// must be active.
template <int X>
__device__ __forceinline__ double quad_xor(double x) {
  static_assert(X >= 1 && X <= 3, "a lane of the same quad");
  // quad_perm selector: lane i of each quad reads lane i ^ X (two bits per lane)
  constexpr int sel = (0 ^ X) | ((1 ^ X) << 2) | ((2 ^ X) << 4) | ((3 ^ X) << 6);
  const unsigned long long b = (unsigned long long)__double_as_longlong(x);
  const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)b, sel, 0xF, 0xF, false);
  const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), sel, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

template <int X>
__device__ __forceinline__ float quad_xor(float x) {
  constexpr int sel = (0 ^ X) | ((1 ^ X) << 2) | ((2 ^ X) << 4) | ((3 ^ X) << 6);
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), sel, 0xF, 0xF, false));
}

// Value of the other lane of the pair (lanes 2p and 2p+1 hold the two sides of one segment).
template <class real>
__device__ __forceinline__ real pair_swap(real x) {
  return quad_xor<1>(x);
}

// STAGE 1: seeds lam_L = dt/2 P + dt Q, lam_Lt = dt^2/8 P + dt^2/6 Q (P = adjoint of W*, Q = of R).
// STAGE 2: seeds lam_Lt = dt^2/3 P (P = adjoint of W^{n+1}) and the adjoint LA of alpha^{n+1}, with
//          the stage's interface DF products DX, DY.
// Thread 2p + s works on side s of interface segment p (s = 0: the cell before the interface).
// RULE >= 0 fixes the hybrid switch rule at compile time (its selects fold away: this kernel is at
// the register limit and pays for every live value); RULE < 0 reads the rule of S at run time.
// The LF 2-interface tile asks for two waves per SIMD (see kAdjShapes).
template <class real, int FLUX, int STAGE, int TF, int TR, int RULE>
__global__ __launch_bounds__(2 * TF * (TR + 4), (FLUX == 0 && TF == 2) ? 2 : 1) void k_adj_faces(
    const real* __restrict__ W, const real* __restrict__ alpha, const real* __restrict__ P,
    const real* __restrict__ Q, const real* __restrict__ LA, const real* __restrict__ DX,
    const real* __restrict__ DY, real* __restrict__ BX, real* __restrict__ BY, GridDesc G, Scheme S,
    const double* __restrict__ dt_hist, int step) {
  using T = AdjTile<TF, TR>;
  __shared__ real sW[4][T::NQ][T::WN];
  __shared__ real sA[T::NQ][T::AN];
  __shared__ real sL[4][2 * TF * T::NQ];  // line values, the two sides of a segment side by side
  __shared__ real sX[5][4][T::NT];         // exchange of line adjoints between rows (m = 0..4)
  __shared__ real sN[4][T::NT];            // each lane's normal-derivative adjoints, parked
  __shared__ real sE[FLUX == 1 ? 22 : 1][T::NT];  // the gas-kinetic reverse's hand-over, parked

  int b = xcd_tile(blockIdx.x, gridDim.x);  // neighbouring tiles share an XCD (and its L2)
  const int nbx = tiles_x<TF, TR>(G.nx, G.ny);
  const int dir = b < nbx ? 0 : 1;
  if (dir) b -= nbx;
  const int nx = G.nx, ny = G.ny;
  const int Nn = dir ? ny : nx, Nt = dir ? nx : ny;
  const int ntf = (Nn + 1 + TF - 1) / TF;
  const int f0 = (b % ntf) * TF, t0 = (b / ntf) * TR;
  const int bcn = dir ? G.bc_y : G.bc_x, bct = dir ? G.bc_x : G.bc_y;
  const real inv_dn = real(dir ? G.inv_dy : G.inv_dx), inv_dt = real(dir ? G.inv_dx : G.inv_dy);
  const size_t N = (size_t)nx * ny;
  const int tid = threadIdx.x;
  const real dt = real(dt_hist[step]);
  const Coef<real> k = make_coef<real, RULE>(S);

  // ---- stage cells (rows t0-4 .. t0+TR+3) and alpha in LDS, local component order; tiles whose halo
  //      lies inside the grid skip the boundary index map (uniform over the workgroup).  Every load is
  //      issued before the first is waited for; threads past the end of a list reload its last entry
  //      (in bounds) and store nothing.
  constexpr int NWE = T::NQ * T::WN, NAE = T::NQ * T::AN;
  constexpr int IW = (NWE + T::NT - 1) / T::NT, IA = (NAE + T::NT - 1) / T::NT;
  const bool inner = f0 - 3 >= 0 && f0 + T::WN - 3 <= Nn && t0 - 4 >= 0 && t0 + T::NQ - 4 <= Nt;
  auto map_n = [&](int i) { return inner ? i : bc_map(i, Nn, bcn); };
  auto map_t = [&](int i) { return inner ? i : bc_map(i, Nt, bct); };
  auto split = [&](int e, int width, int& nl, int& tl) {
    if (dir == 0) {
      tl = e / width;
      nl = e % width;
    } else {
      nl = e / T::NQ;
      tl = e % T::NQ;
    }
  };
  auto gcell = [&](int n, int t) -> size_t { return dir == 0 ? (size_t)t * nx + n : (size_t)n * nx + t; };
  real rw[IW][4], ra[IA];
#pragma unroll
  for (int it = 0; it < IW; ++it) {
    int nl, tl;
    split(min(tid + it * T::NT, NWE - 1), T::WN, nl, tl);
    const size_t g = gcell(map_n(f0 - 3 + nl), map_t(t0 - 4 + tl));
    rw[it][0] = W[g];
    rw[it][1] = W[(dir ? 2 : 1) * N + g];
    rw[it][2] = W[(dir ? 1 : 2) * N + g];
    rw[it][3] = W[3 * N + g];
  }
#pragma unroll
  for (int it = 0; it < IA; ++it) {
    int nl, tl;
    split(min(tid + it * T::NT, NAE - 1), T::AN, nl, tl);
    ra[it] = alpha[gcell(map_n(f0 - 2 + nl), map_t(t0 - 4 + tl))];
  }
  // The seed terms of the cells the segment rows read (the TF+1 cells beside the tile's interfaces,
  // normal index f0-1 .. f0+TF-1, on the NR segment rows), formed once per cell at staging rather
  // than by the four lanes that read each: stage 1 the face-sum adjoints L = dt/2 P + dt Q and
  // Lt = dt^2/8 P + dt^2/6 Q (KS = 8 values per cell); stage 2 Lt = dt^2/3 P and the DF-product
  // adjoints LA (D_n (D_t0 D_t1)) with D_n the product of the cell's face f-1 (it is cell a of
  // interface f) or f+1 (cell b), D_t0, D_t1 those of its two faces across (KS = 6).  Their loads fly
  // with the tile's; the terms wait in the exchange buffer, which is free until the segment reverse.
  // Thread tid < NSC takes one cell; cells off the grid load clamped (unused) entries.
  constexpr int KS = STAGE == 1 ? 8 : 6, NSC = T::NR * (TF + 1);
  static_assert(NSC <= T::NT && KS * NSC <= 20 * T::NT, "seed staging does not fit the tile");
  real* const sS = &sX[0][0][0];
  const int scl = dir == 0 ? tid % (TF + 1) : tid / T::NR, stl = dir == 0 ? tid / (TF + 1) : tid % T::NR;
  real rs[STAGE == 1 ? 8 : 9];
  if (tid < NSC) {
    const int n = min(max(f0 - 1 + scl, 0), Nn - 1), tt = min(max(t0 - 2 + stl, 0), Nt - 1);
    const size_t g = gcell(n, tt), rx = (size_t)nx + 1;
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) rs[kk] = P[kk * N + g];
    if constexpr (STAGE == 1) {
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) rs[4 + kk] = Q[kk * N + g];
    } else {
      rs[4] = LA[g];
      // faces across (x-interfaces: y-faces below, above; y-interfaces: x-faces left, right), then
      // the faces along the normal before and after the cell
      rs[5] = dir == 0 ? DY[(size_t)tt * nx + n] : DX[(size_t)n * rx + tt];
      rs[6] = dir == 0 ? DY[(size_t)(tt + 1) * nx + n] : DX[(size_t)n * rx + tt + 1];
      rs[7] = dir == 0 ? DX[(size_t)tt * rx + n] : DY[(size_t)n * nx + tt];
      rs[8] = dir == 0 ? DX[(size_t)tt * rx + n + 1] : DY[(size_t)(n + 1) * nx + tt];
    }
  }
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
  if (tid < NSC) {  // [term][row][cell]
    real v[KS];
    if constexpr (STAGE == 1) {
      const real h1 = real(0.5) * dt, h2 = dt * dt * real(0.125), r2 = dt * dt * real(1.0 / 6.0);
#pragma unroll
      for (int gc = 0; gc < 4; ++gc) {
        v[gc] = h1 * rs[gc] + dt * rs[4 + gc];
        v[4 + gc] = h2 * rs[gc] + r2 * rs[4 + gc];
      }
    } else {
      const real r3 = dt * dt * real(1.0 / 3.0);
#pragma unroll
      for (int gc = 0; gc < 4; ++gc) v[gc] = r3 * rs[gc];
      const real across = rs[5] * rs[6];
      v[4] = rs[4] * (rs[7] * across);
      v[5] = rs[4] * (rs[8] * across);
    }
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) sS[(kk * T::NR + stl) * (TF + 1) + scl] = v[kk];
  }
  __syncthreads();

  // pair pr = rr * TF + fl in both directions: the TF interfaces of a segment row sit in adjacent
  // lane pairs (one lane quad for TF = 2)
  const int side = tid & 1, pr = tid >> 1;
  const int fl = pr % TF, rr = pr / TF;
  auto lidx = [&](int q, int c) { return q * TF + c; };
  auto pidx = [&](int c, int r) { return r * TF + c; };
  const int f = f0 + fl;
  const int t = t0 - 2 + rr;  // segment row of this pair
  const bool face = f <= Nn;
  const real sgn_dn = side ? -inv_dn : inv_dn;

  // this side's normal stencil on sweep row q (cells ordered away from the far side) and the DF
  // of its cells 1..3
  auto stencil = [&](int q, real(*cs)[4]) {
#pragma unroll
    for (int m = 0; m < 5; ++m)
#pragma unroll
      for (int c = 0; c < 4; ++c) cs[m][c] = sW[c][q][fl + (side ? 5 - m : m)];
  };
  auto a_of = [&](int q, int m) { return sA[q][fl + (side ? 3 - m : m)]; };  // stencil cell m+1
  auto basis_row = [&](int q) {
    real wa[4], wb[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      wa[c] = sW[c][q][fl + 2];
      wb[c] = sW[c][q][fl + 3];
    }
    return make_basis(wa, wb, k);
  };
  auto row_needed = [&](int q) {
    const int tq = t0 - 4 + q;
    return face && tq >= -2 && tq <= Nt + 1;
  };

  // ---- normal sweep (forward), this side: own row q = rr+2, and four extra rows
  //      (q = 0, 1, TR+6, TR+7) on the pairs with rr < 4
  real wn[4] = {0, 0, 0, 0};
  auto ns_row = [&](int q, real* dn) {
    const Basis<real> B = basis_row(q);
    real cs[5][4], w[4];
    stencil(q, cs);
    normal_side<RULE>(B, cs, a_of(q, 0), a_of(q, 1), a_of(q, 2), sgn_dn, k, w, dn);
#pragma unroll
    for (int c = 0; c < 4; ++c) sL[c][2 * lidx(q, fl) + side] = w[c];
  };
  if (row_needed(rr + 2)) ns_row(rr + 2, wn);
  if (rr < 4) {
    const int q2 = rr < 2 ? rr : rr + TR + 4;
    real d[4];
    if (row_needed(q2)) ns_row(q2, d);
  }
  __syncthreads();

  // ---- segment forward, this side: states at the two Gauss points
  const bool seg = face && t >= 0 && t < Nt;
  real al[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) al[q] = sA[rr + 1 + q][fl + 1 + side];
  auto line = [&](int m, int c) -> real { return sL[c][2 * lidx(rr + m, fl) + side]; };
  real gw[2][4], gwt[2][4];
#pragma unroll
  for (int g = 0; g < 2; ++g)
#pragma unroll
    for (int c = 0; c < 4; ++c) gw[g][c] = gwt[g][c] = real(0);
  // the segment's basis is rebuilt from LDS at each use (here, in the segment reverse and in the
  // normal-sweep reverse) rather than held across the phases in between: 20 fewer live values there,
  // 32-48 fewer bytes of spills per lane
  if (seg) segment_side<RULE>(basis_row(rr + 2), line, al, inv_dt, k, gw, gwt);

  // ---- adjoints of the face sums from the cell seeds (face f: -1/dn to cell f-1, +1/dn to cell f)
  const int cmap[4] = {0, dir ? 2 : 1, dir ? 1 : 2, 3};
  real lFs[4] = {0, 0, 0, 0}, lFts[4] = {0, 0, 0, 0}, ldfp = real(0);
  if (seg) {
    const bool has_a = f >= 1, has_b = f < Nn;
    // staged seed terms of cell a = f-1 (cell column fl) and b = f (fl + 1) on this row
    auto sd = [&](int kk, int cl) { return sS[(kk * T::NR + rr) * (TF + 1) + cl]; };
    real lF[4], lFt[4];
    if (STAGE == 1) {
#pragma unroll
      for (int gc = 0; gc < 4; ++gc) {
        const real La = has_a ? sd(gc, fl) : real(0), Lb = has_b ? sd(gc, fl + 1) : real(0);
        const real Lta = has_a ? sd(4 + gc, fl) : real(0), Ltb = has_b ? sd(4 + gc, fl + 1) : real(0);
        lF[gc] = (Lb - La) * inv_dn;
        lFt[gc] = (Ltb - Lta) * inv_dn;
      }
    } else {
#pragma unroll
      for (int gc = 0; gc < 4; ++gc) {
        const real Lta = has_a ? sd(gc, fl) : real(0), Ltb = has_b ? sd(gc, fl + 1) : real(0);
        lF[gc] = real(0);
        lFt[gc] = (Ltb - Lta) * inv_dn;
      }
    }
    // local component order (normal momentum first), quadrature weight 1/2
    lFs[0] = real(0.5) * lF[0];
    lFs[1] = real(0.5) * (dir ? lF[2] : lF[1]);
    lFs[2] = real(0.5) * (dir ? lF[1] : lF[2]);
    lFs[3] = real(0.5) * lF[3];
    lFts[0] = real(0.5) * lFt[0];
    lFts[1] = real(0.5) * (dir ? lFt[2] : lFt[1]);
    lFts[2] = real(0.5) * (dir ? lFt[1] : lFt[2]);
    lFts[3] = real(0.5) * lFt[3];
    // adjoint of the Gauss-point DF product (alpha_new of a cell is the product of its four faces)
    if (STAGE == 2) {
      if (has_a) ldfp += sd(4, fl);
      if (has_b) ldfp += sd(5, fl + 1);
    }
  }

  // ---- Gauss point g = side: both sides' states (the partner's over a lane swap), flux and DF
  //      adjoint there; then each side collects its own state adjoints at both points
  real wl[4], wr[4], wlt[4], wrt[4], wln[4], wrn[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const real mine = side ? gw[1][c] : gw[0][c], mine_t = side ? gwt[1][c] : gwt[0][c];
    const real other = pair_swap(side ? gw[0][c] : gw[1][c]);  // partner's state at my point
    const real other_t = pair_swap(side ? gwt[0][c] : gwt[1][c]);
    const real other_n = pair_swap(wn[c]);
    wl[c] = side ? other : mine;
    wr[c] = side ? mine : other;
    wlt[c] = side ? other_t : mine_t;
    wrt[c] = side ? mine_t : other_t;
    wln[c] = side ? other_n : wn[c];
    wrn[c] = side ? wn[c] : other_n;
  }
  real dfo = real(1);
  if (STAGE == 2 && seg) dfo = df_factor(prim(wl, k), prim(wr, k));
  const real df_other = pair_swap(dfo);
  real lwl[4] = {0, 0, 0, 0}, lwln[4] = {0, 0, 0, 0}, lwlt[4] = {0, 0, 0, 0};
  real lwr[4] = {0, 0, 0, 0}, lwrn[4] = {0, 0, 0, 0}, lwrt[4] = {0, 0, 0, 0};
  const real ldf = STAGE == 2 ? ldfp * df_other : real(0);
  if constexpr (FLUX == 0) {
    if (seg) gp_flux_adj<real, FLUX>(wl, wln, wlt, wr, wrn, wrt, dt, k, lFs, lFts, ldf, lwl, lwln, lwlt, lwr, lwrn, lwrt);
  } else {
    // The gas-kinetic reverse in two halves around a barrier: the Gauss point's 24 states and the 22
    // values handed from the equilibrium-state reverse to the side reverse wait in the lane's own
    // LDS slots (the exchange buffers hold nothing else between the seeds and the segment reverse),
    // so that neither half holds the other's live values; the barrier makes the compiler reload them.
    GksEqAdj<real> e{};
    if (seg) gks_flux_adj_eq(wln, wlt, wrn, wrt, prim(wl, k), prim(wr, k), dt, k, lFs, lFts, e);
    __syncthreads();  // every lane has read its staged seeds from the exchange buffer
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      sX[0][c][tid] = wl[c];
      sX[1][c][tid] = wr[c];
      sX[2][c][tid] = wln[c];
      sX[3][c][tid] = wrn[c];
      sX[4][c][tid] = wlt[c];
      sN[c][tid] = wrt[c];
      sE[c][tid] = e.lWc[c];
      sE[4 + c][tid] = e.lWcn[c];
      sE[8 + c][tid] = e.lWct[c];
      sE[12 + c][tid] = e.lFlr[c];
      sE[16 + c][tid] = e.lMalr[c];
    }
    sE[20][tid] = e.lpl;
    sE[21][tid] = e.lpr;
    __syncthreads();
    if (seg) {
      real vl[4], vr[4], vln[4], vrn[4], vlt[4], vrt[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        vl[c] = sX[0][c][tid];
        vr[c] = sX[1][c][tid];
        vln[c] = sX[2][c][tid];
        vrn[c] = sX[3][c][tid];
        vlt[c] = sX[4][c][tid];
        vrt[c] = sN[c][tid];
        e.lWc[c] = sE[c][tid];
        e.lWcn[c] = sE[4 + c][tid];
        e.lWct[c] = sE[8 + c][tid];
        e.lFlr[c] = sE[12 + c][tid];
        e.lMalr[c] = sE[16 + c][tid];
      }
      e.lpl = sE[20][tid];
      e.lpr = sE[21][tid];
      const Prim<real> ql = prim(vl, k), qr = prim(vr, k);
      PrimAdj<real> lql, lqr;
      lql.zero();
      lqr.zero();
      gks_flux_adj_sides(vln, vlt, vrn, vrt, ql, qr, k, e, lwln, lwlt, lwrn, lwrt, lql, lqr);
      df_factor_adj(ql, qr, ldf, lql, lqr);
      prim_adj(vl, ql, k, lql, lwl);
      prim_adj(vr, qr, k, lqr, lwr);
    }
  }
  real lgw[2][4], lgwt[2][4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const real own = side ? lwr[c] : lwl[c], own_t = side ? lwrt[c] : lwlt[c], own_n = side ? lwrn[c] : lwln[c];
    const real got = pair_swap(side ? lwl[c] : lwr[c]);  // my side's adjoint at the partner's point
    const real got_t = pair_swap(side ? lwlt[c] : lwrt[c]);
    const real got_n = pair_swap(side ? lwln[c] : lwrn[c]);
    lgw[0][c] = side ? got : own;
    lgw[1][c] = side ? own : got;
    lgwt[0][c] = side ? got_t : own_t;
    lgwt[1][c] = side ? own_t : got_t;
    // Gauss point 0 first on both lanes; parked in the lane's own LDS slots until the normal-sweep
    // reverse instead of being held (and spilled) through the segment reverse
    sN[c][tid] = side ? got_n + own_n : own_n + got_n;
  }
  __syncthreads();  // the reverse reloads its LDS inputs after this point

  // ---- segment reverse, this side: characteristic line adjoints, then the line adjoints of the
  //      five rows each segment reads, summed per row through LDS in a fixed order
  //      In two halves: the reverse of the Gauss-point reconstruction, one characteristic component
  //      at a time, parks the components' line adjoints in the lane's own slots of the exchange
  //      buffer ([row][component]); after a barrier, which makes the compiler reload them rather
  //      than hold 20 values through all four components, the projection's reverse turns each row's
  //      four into that row's line adjoints in the same slots.
  BasisAdj<real> lB;
  lB.zero();
  real la_seg = real(0);
  if (seg)
    segment_side_adj_q<RULE>(basis_row(rr + 2), line, al, inv_dt, k, lgw, lgwt,
                             [&](int C, int m, real v) { sX[m][C][tid] = v; }, lB, la_seg);
  __syncthreads();
  if (seg) {
    const Basis<real> B = basis_row(rr + 2);
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      real w[4], lq[4], d[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        w[c] = line(m, c);
        lq[c] = sX[m][c][tid];
      }
      segment_side_adj_line(B, w, lq, d, lB);
#pragma unroll
      for (int c = 0; c < 4; ++c) sX[m][c][tid] = d[c];
    }
  } else {
#pragma unroll
    for (int m = 0; m < 5; ++m)
#pragma unroll
      for (int c = 0; c < 4; ++c) sX[m][c][tid] = real(0);
  }
  __syncthreads();
  real acc[4] = {0, 0, 0, 0};
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    const int src = rr + 2 - m;  // the segment whose line m is this pair's row
    if (src >= 0 && src < T::NR) {
      const int st = 2 * pidx(fl, src) + side;
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[c] += sX[m][c][st];
    }
  }

  // ---- normal-sweep adjoint of the rows this tile owns: its TR rows, the two ghost rows below the
  //      grid (first tile) and the two above it (tile of the last row)
  const bool own = face && ((rr >= 2 && rr < TR + 2 && t < Nt) || (t0 == 0 && t < 0) ||
                            (t >= Nt && t <= Nt + 1 && t0 + TR >= Nt));
  real lcs[5][4];
#pragma unroll
  for (int m = 0; m < 5; ++m)
#pragma unroll
    for (int c = 0; c < 4; ++c) lcs[m][c] = real(0);
  real la_ns = real(0);
  if (own) {
    auto cell = [&](int m, int c) -> real { return sW[c][rr + 2][fl + (side ? 5 - m : m)]; };
    auto lc_add = [&](int m, int c, real v) { lcs[m][c] += v; };
    real lwn[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) lwn[c] = sN[c][tid];
    normal_side_adj<RULE>(basis_row(rr + 2), cell, a_of(rr + 2, 0), a_of(rr + 2, 1), a_of(rr + 2, 2), sgn_dn, k, acc,
                          lwn, lc_add, lB, la_ns);
  }
  // basis adjoint of the pair (side 0 first on both lanes), then the two cells it is built from
  BasisAdj<real> lBt;
  {
    BasisAdj<real> o;
    o.u = pair_swap(lB.u);
    o.v = pair_swap(lB.v);
    o.c = pair_swap(lB.c);
    o.ic = pair_swap(lB.ic);
    o.H = pair_swap(lB.H);
    o.hq2 = pair_swap(lB.hq2);
    o.b1 = pair_swap(lB.b1);
    o.b2 = pair_swap(lB.b2);
    if (side) {
      lBt = o;
      basis_adj_add(lBt, lB);
    } else {
      lBt = lB;
      basis_adj_add(lBt, o);
    }
  }
  // cells f-2+... : side 0 holds stencil cells 0..4 (lcs[m] = cell m), side 1 cells 5..1
  // (lcs[m] = cell 5-m).  Lane 0 of a pair forms cells 0, 1, 2 and the DF of cell f-1; lane 1 cells
  // 3, 4, 5 and the DF of cell f.  Each lane needs the partner's lcs[3] and lcs[4].
  real r3[4], r4[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    r3[c] = pair_swap(lcs[3][c]);
    r4[c] = pair_swap(lcs[4][c]);
  }
  real out[3][4], dfv = real(0);
#pragma unroll
  for (int m = 0; m < 3; ++m)
#pragma unroll
    for (int c = 0; c < 4; ++c) out[m][c] = real(0);
  if (own) {
    real lbc[4] = {0, 0, 0, 0}, lbc2[4] = {0, 0, 0, 0};
    {
      real wa[4], wb[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        wa[c] = sW[c][rr + 2][fl + 2];
        wb[c] = sW[c][rr + 2][fl + 3];
      }
      make_basis_adj(wa, wb, k, lBt, lbc, lbc2);  // the same adjoint reaches both cells
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      if (side == 0) {
        out[0][c] = lcs[0][c];
        out[1][c] = lcs[1][c] + r4[c];
        out[2][c] = (lcs[2][c] + r3[c]) + lbc[c];
      } else {
        out[0][c] = (r3[c] + lcs[2][c]) + lbc[c];
        out[1][c] = r4[c] + lcs[1][c];
        out[2][c] = lcs[0][c];
      }
    }
    dfv = la_seg + la_ns;
  }
  // The tile's two interfaces of this row (lanes q = 0, 1: interface f0, sides 0, 1; q = 2, 3:
  // interface f0+1) read overlapping stencils, cells f0-3 .. f0+2 and f0-2 .. f0+3: their cell
  // adjoints are summed here into the row's window of seven cells w = 0..6 (cell f0-3+w) and three
  // DF values d = 0..2 (cell f0-1+d), interface f0's term first; lanes that own no segment (rows
  // outside the tile, an interface past the grid) add zeros.  With A = interface f0, B = f0+1 and
  // [m] the m-th cell a side forms: lane q = side s of A writes w = 3s + m = A_s[m] + (B_s[m-1] for
  // m = 1, 2; B_0[2] for s = 1, m = 0) and d = s = A_s + (B_0 for s = 1), the same code on both
  // lanes; lane 3 writes w = 6 = B_1[2] and d = 2 = B_1.
  static_assert(TF == 2, "the window of a tile row covers two interfaces");
  real x2[2][4], x3[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    x2[0][c] = quad_xor<2>(out[0][c]);  // B_s on lane s (A's lanes)
    x2[1][c] = quad_xor<2>(out[1][c]);
    x3[c] = quad_xor<3>(out[2][c]);  // B_0[2] on lane 1
  }
  const real df3 = quad_xor<3>(dfv);                     // B_0's DF value on lane 1
  const float own_a = quad_xor<2>(own ? 1.0f : 0.0f);   // on B's lanes: whether A owns the row
  const bool row_own = fl == 0 ? own : own_a != 0.0f;
  if (!row_own || (fl == 1 && side == 0)) return;
  size_t sB, wfs, wrs;
  real* o;
  const int kt = f0 / TF;
  if (dir == 0) {
    const size_t nk = (size_t)(nx + 2) / 2;
    sB = (size_t)(ny + 4) * nk;
    wfs = 1;
    wrs = nk;
    o = BX;
  } else {
    const size_t nk = (size_t)(ny + 2) / 2;
    sB = nk * (nx + 4);
    wfs = (size_t)nx + 4;
    wrs = 1;
    o = BY;
  }
  o += (size_t)kt * wfs + (size_t)(t + 2) * wrs;
  if (fl == 0) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      o[((3 * side) * 4 + cmap[c]) * sB] = out[0][c] + (side ? x3[c] : real(0));
      o[((3 * side + 1) * 4 + cmap[c]) * sB] = out[1][c] + x2[0][c];
      o[((3 * side + 2) * 4 + cmap[c]) * sB] = out[2][c] + x2[1][c];
    }
    o[(28 + side) * sB] = dfv + (side ? df3 : real(0));
  } else {
#pragma unroll
    for (int c = 0; c < 4; ++c) o[(6 * 4 + cmap[c]) * sB] = out[2][c];
    o[30 * sB] = dfv;
  }
}

// Indices in [lo, hi] that the boundary map sends to cell n of a line of Nn cells: a contiguous
// range for transmissive boundaries, a stride-Nn progression for periodic ones.
struct Preimages {
  int first, stride, last;
};

__device__ __forceinline__ Preimages preimages(int n, int Nn, int bc, int lo, int hi) {
  Preimages p;
  if (bc == DFW_BC_PERIODIC) {
    p.first = lo + (n - lo) % Nn;
    p.stride = Nn;
    p.last = hi;
  } else {
    p.first = n == 0 ? lo : n;
    p.last = n == Nn - 1 ? hi : n;
    p.stride = 1;
  }
  return p;
}

// Sum of the window-buffer entries of one direction that belong to cell (n, t) (normal, tangential
// index).  The window of tile k (interfaces 2k and 2k+1) and row `row` holds, at slot w*4 + c, the
// adjoint of component c of cell 2k-3+w (w = 0..6), and at slot 28 + d that of the DF of cell
// 2k-1+d (d = 0..2); it sits at B[slot*sB + k*fs + (row+2)*rs].  A cell is in the windows of three or
// four tiles (its DF in one or two), summed in increasing k.
template <class real>
__device__ __forceinline__ void gather_dir(const real* __restrict__ B, size_t sB, size_t fs, size_t rs, int n, int Nn,
                                           int bcn, int t, int Nt, int bct, real* g, real& ga) {
  const int nk = (Nn + 2) / 2;
  const Preimages pt = preimages(t, Nt, bct, -2, Nt + 1);
  const Preimages pn = preimages(n, Nn, bcn, -3, Nn + 2);
  for (int tp = pt.first; tp <= pt.last; tp += pt.stride) {
    const real* row = B + (size_t)(tp + 2) * rs;
    for (int e = pn.first; e <= pn.last; e += pn.stride) {
      const int k0 = max((e - 2) >> 1, 0), k1 = min((e + 3) >> 1, nk - 1);  // floor division
      for (int kk = k0; kk <= k1; ++kk) {
        const int w = e - 2 * kk + 3;
#pragma unroll
        for (int c = 0; c < 4; ++c) g[c] += row[(w * 4 + c) * sB + kk * fs];
      }
      const int d0 = max(e >> 1, 0), d1 = min((e + 1) >> 1, nk - 1);
      for (int kk = d0; kk <= d1; ++kk) ga += row[(28 + e - 2 * kk + 1) * sB + kk * fs];
    }
  }
}

// STAGE 2: LWs = adjoint of W* (from the stage-2 interfaces), LA = stage-2 part of the adjoint of
//          alpha^n.
// STAGE 1: LW <- LW + LWs + stage-1 part (adjoint of W^n), LA <- LA + stage-1 part.
template <class real, int STAGE>
__global__ __launch_bounds__(kCellBlock) void k_adj_gather(const real* __restrict__ BX, const real* __restrict__ BY,
                                                           real* __restrict__ LW, real* __restrict__ LWs,
                                                           real* __restrict__ LA, GridDesc G) {
  const int nx = G.nx, ny = G.ny;
  const size_t N = (size_t)nx * ny, o = (size_t)blockIdx.x * kCellBlock + threadIdx.x;
  if (o >= N) return;
  const int i = (int)(o % nx), j = (int)(o / nx);
  real g[4] = {0, 0, 0, 0}, ga = 0;
  const size_t nkx = (size_t)(nx + 2) / 2, nky = (size_t)(ny + 2) / 2;
  gather_dir(BX, (size_t)(ny + 4) * nkx, 1, nkx, i, nx, G.bc_x, j, ny, G.bc_y, g, ga);
  gather_dir(BY, nky * (nx + 4), (size_t)nx + 4, 1, j, ny, G.bc_y, i, nx, G.bc_x, g, ga);
  if (STAGE == 2) {
#pragma unroll
    for (int c = 0; c < 4; ++c) LWs[c * N + o] = g[c];
    LA[o] = ga;
  } else {
#pragma unroll
    for (int c = 0; c < 4; ++c) LW[c * N + o] = LW[c * N + o] + LWs[c * N + o] + g[c];
    LA[o] = LA[o] + ga;
  }
}

__global__ void k_set_dt(Ctrl* ctrl, const double* __restrict__ dt_hist, int step) {
  if (threadIdx.x == 0 && blockIdx.x == 0) ctrl->dt = dt_hist[step];
}

template <class real>
__global__ __launch_bounds__(kCellBlock) void k_fill(real* __restrict__ x, real v, size_t n) {
  const size_t o = (size_t)blockIdx.x * kCellBlock + threadIdx.x;
  if (o < n) x[o] = v;
}

// ------------------------------------------------------------------------------------------------
// Host side.
// ------------------------------------------------------------------------------------------------
struct AdjShape {
  int tf, tr;
};
// Interface tiles of the adjoint kernel, per flux (LF, GKS): 2 interfaces x 60 rows, 256 threads.
// The 60-row tile recomputes the segment adjoint (the costly part, above all with the GKS flux) for
// 64 segment rows per 60 owned.  The LF kernel is held to two waves per SIMD (launch bounds), so that
// two workgroups share a compute unit and one's barriers and staging overlap the other's arithmetic;
// the GKS kernel needs one wave per SIMD with its accumulation registers as well, and 121 KB of LDS.
static constexpr AdjShape kAdjShapes[2] = {{2, 60}, {2, 60}};

static int adj_tiles(int flux, int nx, int ny) {
  const AdjShape s = kAdjShapes[flux];
  return ((nx + 1 + s.tf - 1) / s.tf) * ((ny + s.tr - 1) / s.tr) + ((ny + 1 + s.tf - 1) / s.tf) * ((nx + s.tr - 1) / s.tr);
}

template <class real, int FLUX, int STAGE>
static void launch_adj_faces(const real* W, const real* A, const real* P, const real* Q, const real* LA,
                             const real* DX, const real* DY, real* BX, real* BY, const GridDesc& G, const Scheme& S,
                             const double* dt_hist, int step, hipStream_t st) {
  constexpr int TF = kAdjShapes[FLUX].tf, TR = kAdjShapes[FLUX].tr;
  if (S.sw == 0)  // the switch of eq. (42) as printed
    hipLaunchKernelGGL((k_adj_faces<real, FLUX, STAGE, TF, TR, 0>), dim3(adj_tiles(FLUX, G.nx, G.ny)),
                       dim3(2 * TF * (TR + 4)), 0, st, W, A, P, Q, LA, DX, DY, BX, BY, G, S, dt_hist, step);
  else
    hipLaunchKernelGGL((k_adj_faces<real, FLUX, STAGE, TF, TR, -1>), dim3(adj_tiles(FLUX, G.nx, G.ny)),
                       dim3(2 * TF * (TR + 4)), 0, st, W, A, P, Q, LA, DX, DY, BX, BY, G, S, dt_hist, step);
}

// Checkpoint store: one slot per segment of ckpt_every steps, slot = W (4N) | alpha (N).  With a
// checkpoint at every step (ckpt_every = 1) the slot is the whole record of its step, W^n | alpha^n |
// W* | stage-2 DF products of the x and the y interfaces, and the adjoint recomputes nothing.
struct CkptLayout {
  size_t w_off, a_off, ws_off, dfx_off, dfy_off, slot, total;
  bool tape;
};

static CkptLayout ckpt_layout(const dfw_grid* g, size_t es, int nsteps, int every) {
  CkptLayout L;
  const size_t N = (size_t)g->nx * g->ny;
  const size_t sx = (size_t)g->ny * (g->nx + 1), sy = (size_t)(g->ny + 1) * g->nx;
  L.tape = every == 1;
  L.w_off = 0;
  L.a_off = align256(4 * N * es);
  L.slot = L.a_off + align256(N * es);
  L.ws_off = L.dfx_off = L.dfy_off = 0;
  if (L.tape) {
    L.ws_off = L.slot;
    L.dfx_off = L.ws_off + align256(4 * N * es);
    L.dfy_off = L.dfx_off + align256(sx * es);
    L.slot = L.dfy_off + align256(sy * es);
  }
  const int nseg = nsteps > 0 ? (nsteps + every - 1) / every : 0;
  L.total = (size_t)nseg * L.slot;
  return L;
}

// Adjoint workspace: forward workspace | states of one segment | adjoint cells | window buffers.
struct AdjLayout {
  WsLayout fwd;
  size_t wst, ast, wss, dfx, dfy, lw, lws, la, bx, by, total;
  size_t wN, aN, sx, sy;  // element strides of one step's W, alpha and DF planes
};

static AdjLayout adj_layout(const dfw_grid* g, size_t es, int every) {
  AdjLayout L;
  L.fwd = layout(g, es);
  const size_t N = (size_t)g->nx * g->ny;
  const size_t sx = (size_t)g->ny * (g->nx + 1), sy = (size_t)(g->ny + 1) * g->nx;
  if (every == 1) every = 0;  // the checkpoint store holds every step's record: nothing is recomputed
  L.wN = align256(4 * N * es) / es;
  L.aN = align256(N * es) / es;
  L.sx = align256(sx * es) / es;
  L.sy = align256(sy * es) / es;
  size_t off = L.fwd.total;
  L.wst = off;  // W^n of every step of a segment (the first comes from the checkpoint)
  off += (size_t)every * L.wN * es;
  L.ast = off;
  off += (size_t)every * L.aN * es;
  L.wss = off;  // W* of every step
  off += (size_t)every * L.wN * es;
  L.dfx = off;  // stage-2 interface DF products of every step
  off += (size_t)every * L.sx * es;
  L.dfy = off;
  off += (size_t)every * L.sy * es;
  L.lw = off;
  off = align256(off + 4 * N * es);
  L.lws = off;
  off = align256(off + 4 * N * es);
  L.la = off;
  off = align256(off + N * es);
  L.bx = off;  // window buffers: kAdjSlots slots x rows x tiles of two interfaces
  off = align256(off + (size_t)kAdjSlots * (g->ny + 4) * ((g->nx + 2) / 2) * es);
  L.by = off;
  off = align256(off + (size_t)kAdjSlots * ((g->ny + 2) / 2) * (g->nx + 4) * es);
  L.total = off;
  return L;
}

// Forward steps with checkpoints: the ordinary enqueue with a copy of (W, alpha) into slot n/every
// before every step n that starts a segment; with ckpt_every = 1 also the W* and the stage-2 DF
// products of step n (still in the workspace until step n + 1 starts) into slot n.
template <class real>
static dfw_status run_ckpt_impl(real* W, real* A, const dfw_grid* g, const dfw_params* p, int nsteps, int every,
                                char* ckpt, char* ws, double* dt_hist, double* t_out, int32_t* fail_step,
                                hipStream_t st) {
  const size_t es = sizeof(real);
  const size_t N = (size_t)g->nx * g->ny;
  WsLayout L = layout(g, es);
  CkptLayout C = ckpt_layout(g, es, nsteps, every);
  Ctrl* ctrl = (Ctrl*)(ws + L.ctrl_off);
  const GridDesc G = make_desc(g);
  const size_t sx = (size_t)g->ny * (g->nx + 1), sy = (size_t)(g->ny + 1) * g->nx;
  auto record = [&](int n) -> hipError_t {  // tape: the intermediates of step n
    char* slot = ckpt + (size_t)n * C.slot;
    hipError_t e = hipMemcpyAsync(slot + C.ws_off, ws + L.ws_off, 4 * N * es, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(slot + C.dfx_off, ws + L.fx_off + 8 * sx * es, sx * es, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(slot + C.dfy_off, ws + L.fy_off + 8 * sy * es, sy * es, hipMemcpyDeviceToDevice, st);
    return e;
  };
  auto hook = [&](int n) -> hipError_t {
    if (C.tape && n > 0) {
      hipError_t e = record(n - 1);
      if (e != hipSuccess) return e;
    }
    if (n % every) return hipSuccess;
    char* slot = ckpt + (size_t)(n / every) * C.slot;
    hipError_t e = hipMemcpyAsync(slot + C.w_off, W, 4 * N * es, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(slot + C.a_off, A, N * es, hipMemcpyDeviceToDevice, st);
    return e;
  };
  hipError_t he = hipSuccess;
  enqueue_steps<real>(W, A, (real*)(ws + L.ws_off), (real*)(ws + L.r_off), (real*)(ws + L.fx_off),
                      (real*)(ws + L.fy_off), ctrl, 1, G, nullptr, nullptr, shape_tiles(p->tile, g->nx, g->ny),
                      nullptr, (int)cell_blocks(G), p, nsteps, dt_hist, st, [&](int n) {
                        if (he == hipSuccess) he = hook(n);
                      });
  if (he == hipSuccess && C.tape && nsteps > 0) he = record(nsteps - 1);
  HIP_TRY(he);
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

template <class real, int FLUX>
static dfw_status adjoint_impl(const dfw_grid* g, const dfw_params* p, int nsteps, int every, const char* ckpt,
                               const double* dt_hist, const real* gW_final, const real* gA_final, real* gW0,
                               real* gA0, char* ws, hipStream_t st) {
  const size_t es = sizeof(real);
  const size_t N = (size_t)g->nx * g->ny;
  const AdjLayout L = adj_layout(g, es, every);
  const CkptLayout C = ckpt_layout(g, es, nsteps, every);
  const GridDesc G = make_desc(g);
  const Scheme S = make_scheme(p);
  Ctrl* ctrl = (Ctrl*)(ws + L.fwd.ctrl_off);
  real* R = (real*)(ws + L.fwd.r_off);
  real* FX = (real*)(ws + L.fwd.fx_off);
  real* FY = (real*)(ws + L.fwd.fy_off);
  real* LW = (real*)(ws + L.lw);
  real* LWs = (real*)(ws + L.lws);
  real* LA = (real*)(ws + L.la);
  real* BX = (real*)(ws + L.bx);
  real* BY = (real*)(ws + L.by);
  auto Wst = [&](int l) { return (real*)(ws + L.wst) + (size_t)l * L.wN; };
  auto Ast = [&](int l) { return (real*)(ws + L.ast) + (size_t)l * L.aN; };
  auto Wss = [&](int l) { return (real*)(ws + L.wss) + (size_t)l * L.wN; };
  auto DFX = [&](int l) { return (real*)(ws + L.dfx) + (size_t)l * L.sx; };
  auto DFY = [&](int l) { return (real*)(ws + L.dfy) + (size_t)l * L.sy; };
  const size_t sx = (size_t)g->ny * (g->nx + 1), sy = (size_t)(g->ny + 1) * g->nx;
  const unsigned nb = cell_blocks(G);

  FaceLaunch FL;
  FL.shape = p->tile;
  FL.flux = FLUX;
  FL.nblocks = shape_tiles(p->tile, g->nx, g->ny);
  FL.tiles = nullptr;
  FL.grids = nullptr;
  FL.G0 = G;
  FL.ctrls = ctrl;
  FL.S = S;
  FL.dt_host = 0.0;
  FL.lead = 0;  // dt from the control block, set from dt_hist before every step
  FL.nsteps = nsteps;
  FL.dt_hist = nullptr;

  hipLaunchKernelGGL(k_ctrl_init, dim3(1), dim3(64), 0, st, ctrl, 1);
  HIP_TRY(hipMemcpyAsync(LW, gW_final, 4 * N * es, hipMemcpyDeviceToDevice, st));
  if (gA_final) HIP_TRY(hipMemcpyAsync(LA, gA_final, N * es, hipMemcpyDeviceToDevice, st));
  else hipLaunchKernelGGL(k_fill<real>, dim3(nb), dim3(kCellBlock), 0, st, LA, real(0), N);

  const int nseg = (nsteps + every - 1) / every;
  for (int s = nseg - 1; s >= 0; --s) {
    const int n0 = s * every, n1 = std::min(nsteps, n0 + every);
    const char* slot = ckpt + (size_t)s * C.slot;
    const real* W0 = (const real*)(slot + C.w_off);
    const real* A0 = (const real*)(slot + C.a_off);
    auto Wn = [&](int l) { return l == 0 ? W0 : (const real*)Wst(l); };
    auto An = [&](int l) { return l == 0 ? A0 : (const real*)Ast(l); };
    if (C.tape) {  // one step, recorded whole by the forward run: reverse it directly
      real* Wsl = (real*)(slot + C.ws_off);
      real* DXl = (real*)(slot + C.dfx_off);
      real* DYl = (real*)(slot + C.dfy_off);
      timed(DFW_K_ADJ_FACES2, st, [&] {
        launch_adj_faces<real, FLUX, 2>(Wsl, A0, LW, nullptr, LA, DXl, DYl, BX, BY, G, S, dt_hist, n0, st);
      });
      timed(DFW_K_ADJ_GATHER, st, [&] {
        hipLaunchKernelGGL((k_adj_gather<real, 2>), dim3(nb), dim3(kCellBlock), 0, st, BX, BY, LW, LWs, LA, G);
      });
      timed(DFW_K_ADJ_FACES1, st, [&] {
        launch_adj_faces<real, FLUX, 1>(W0, A0, LWs, LW, nullptr, nullptr, nullptr, BX, BY, G, S, dt_hist, n0, st);
      });
      timed(DFW_K_ADJ_GATHER, st, [&] {
        hipLaunchKernelGGL((k_adj_gather<real, 1>), dim3(nb), dim3(kCellBlock), 0, st, BX, BY, LW, LWs, LA, G);
      });
      continue;
    }
    // recompute the segment, keeping W^n, alpha^n, W* and the stage-2 DF products of every step
    for (int n = n0; n < n1; ++n) {
      const int l = n - n0;
      hipLaunchKernelGGL(k_set_dt, dim3(1), dim3(64), 0, st, ctrl, dt_hist, n);
      FL.step = n;
      FL.out = OUT_F | OUT_FT;
      timed(DFW_K_FACES1, st, [&] { launch_faces<real>(FL, Wn(l), An(l), FX, FY, st); });
      timed(DFW_K_UPDATE1, st, [&] {
        hipLaunchKernelGGL(k_update1<real>, dim3(nb), dim3(kCellBlock), 0, st, Wn(l), FX, FY, Wss(l), R, ctrl, G,
                           nullptr, nullptr, n, 0);
      });
      FL.out = OUT_FT | OUT_DF;
      timed(DFW_K_FACES2, st, [&] { launch_faces<real>(FL, Wss(l), An(l), FX, FY, st); });
      HIP_TRY(hipMemcpyAsync(DFX(l), FX + 8 * sx, sx * es, hipMemcpyDeviceToDevice, st));
      HIP_TRY(hipMemcpyAsync(DFY(l), FY + 8 * sy, sy * es, hipMemcpyDeviceToDevice, st));
      if (n + 1 < n1)
        timed(DFW_K_UPDATE2, st, [&] {
          hipLaunchKernelGGL(k_update2<real>, dim3(nb), dim3(kCellBlock), 0, st, Wst(l + 1), Ast(l + 1), R, FX, FY,
                             ctrl, G, nullptr, nullptr, S, n);
        });
    }
    // reverse the steps of the segment
    for (int n = n1 - 1; n >= n0; --n) {
      const int l = n - n0;
      timed(DFW_K_ADJ_FACES2, st, [&] {
        launch_adj_faces<real, FLUX, 2>(Wss(l), An(l), LW, nullptr, LA, DFX(l), DFY(l), BX, BY, G, S, dt_hist, n, st);
      });
      timed(DFW_K_ADJ_GATHER, st, [&] {
        hipLaunchKernelGGL((k_adj_gather<real, 2>), dim3(nb), dim3(kCellBlock), 0, st, BX, BY, LW, LWs, LA, G);
      });
      timed(DFW_K_ADJ_FACES1, st, [&] {
        launch_adj_faces<real, FLUX, 1>(Wn(l), An(l), LWs, LW, nullptr, nullptr, nullptr, BX, BY, G, S, dt_hist, n,
                                        st);
      });
      timed(DFW_K_ADJ_GATHER, st, [&] {
        hipLaunchKernelGGL((k_adj_gather<real, 1>), dim3(nb), dim3(kCellBlock), 0, st, BX, BY, LW, LWs, LA, G);
      });
    }
  }
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(gW0, LW, 4 * N * es, hipMemcpyDeviceToDevice, st));
  if (gA0) HIP_TRY(hipMemcpyAsync(gA0, LA, N * es, hipMemcpyDeviceToDevice, st));
  Ctrl h;
  HIP_TRY(hipMemcpyAsync(&h, ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (h.fail_at != kNoFail) return fail(DFW_ENONPHYS, "non-physical state while recomputing the forward steps");
  return DFW_OK;
}

}  // namespace dfw
