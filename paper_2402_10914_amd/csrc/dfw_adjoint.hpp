// Hand-written reverse-mode (adjoint) counterparts of the device arithmetic in dfw_math.hpp.
//
// Convention: for y = f(x), f_adj(x, ..., ly, lx) adds (dy/dx)^T ly into lx (accumulates; callers
// zero the adjoint arrays).  Each adjoint recomputes the forward intermediates it needs from the
// primal inputs.  Kinks follow a fixed subgradient convention: d|x| = sign(x) with sign(0) = 0;
// max(a, b) routes to a when a >= b; the hybrid switch of eq. (42) has zero derivative (the branch
// taken is differentiated); dt is held fixed.
#pragma once

#include "dfw_math.hpp"

namespace dfw {

template <class real>
DFW_HD real sgn(real x) {
  return x > real(0) ? real(1) : (x < real(0) ? real(-1) : real(0));
}

// ------------------------------------------------------------------------------------------------
// Characteristic basis.
// ------------------------------------------------------------------------------------------------
template <class real>
struct BasisAdj {
  real u, v, c, ic, H, hq2, b1, b2;
  DFW_HD void zero() { u = v = c = ic = H = hq2 = b1 = b2 = real(0); }
};

template <class real>
DFW_HD void make_basis_adj(const real* wa, const real* wb, const Coef<real>& k, const BasisAdj<real>& lB, real* lwa,
                           real* lwb) {
  const real h = real(0.5);
  real r = h * (wa[0] + wb[0]), m = h * (wa[1] + wb[1]), n = h * (wa[2] + wb[2]), e = h * (wa[3] + wb[3]);
  real ir = real(1) / r;
  real u = m * ir, v = n * ir;
  real hq2 = h * (u * u + v * v);
  real p = k.gm1 * (e - r * hq2);
  real c2 = k.gamma * p * ir;
  real c = sqrt(c2);
  real ic = real(1) / c;
  real b1 = k.gm1 / c2;
  real l_hq2 = lB.hq2 + lB.b2 * b1;
  real l_b1 = lB.b1 + lB.b2 * hq2;
  real l_c2 = -l_b1 * b1 / c2;
  real l_e = lB.H * ir, l_p = lB.H * ir, l_ir = lB.H * (e + p);
  real l_c = lB.c - lB.ic * ic * ic;
  l_c2 += l_c * real(0.5) / c;
  l_p += l_c2 * k.gamma * ir;
  l_ir += l_c2 * k.gamma * p;
  l_e += l_p * k.gm1;
  real l_r = -l_p * k.gm1 * hq2;
  l_hq2 += -l_p * k.gm1 * r;
  real l_u = lB.u + l_hq2 * u, l_v = lB.v + l_hq2 * v;
  real l_m = l_u * ir, l_n = l_v * ir;
  l_ir += l_u * m + l_v * n;
  l_r += -l_ir * ir * ir;
  real lw[4] = {h * l_r, h * l_m, h * l_n, h * l_e};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    lwa[i] += lw[i];
    lwb[i] += lw[i];
  }
}

template <class real>
DFW_HD void project_adj(const Basis<real>& B, const real* w, const real* lq, real* lw, BasisAdj<real>& lB) {
  const real h = real(0.5);
  real lT = h * lq[0] - lq[1] + h * lq[3];
  real ls = h * lq[0] - h * lq[3];
  lw[0] += lq[1] - B.v * lq[2];
  lw[2] += lq[2];
  lB.v += -w[0] * lq[2];
  // s = (u w0 - w1) ic
  lB.u += ls * w[0] * B.ic;
  lw[0] += ls * B.u * B.ic;
  lw[1] += -ls * B.ic;
  lB.ic += ls * (B.u * w[0] - w[1]);
  // T = b2 w0 - b1 X, X = u w1 + v w2 - w3
  real X = B.u * w[1] + B.v * w[2] - w[3];
  lB.b2 += lT * w[0];
  lw[0] += lT * B.b2;
  lB.b1 += -lT * X;
  real lX = -lT * B.b1;
  lB.u += lX * w[1];
  lw[1] += lX * B.u;
  lB.v += lX * w[2];
  lw[2] += lX * B.v;
  lw[3] += -lX;
}

// unproject_adj in two parts: lq += R^T lw does not depend on q; the basis part does.
template <class real>
DFW_HD void unproject_adj_q(const Basis<real>& B, const real* lw, real* lq) {
  real lw0 = lw[0] + B.u * lw[1] + B.v * lw[2];
  real ldq = B.c * lw[1] + B.u * B.c * lw[3];
  lq[0] += lw0 - ldq + lw[3] * B.H;
  lq[1] += lw0 + lw[3] * B.hq2;
  lq[2] += lw[2] + lw[3] * B.v;
  lq[3] += lw0 + ldq + lw[3] * B.H;
}

template <class real>
DFW_HD void unproject_adj_B(const Basis<real>& B, const real* q, const real* lw, BasisAdj<real>& lB) {
  real w0 = q[0] + q[1] + q[3];
  real dq = q[3] - q[0];
  lB.u += lw[1] * w0 + lw[3] * B.c * dq;
  lB.c += lw[1] * dq + lw[3] * B.u * dq;
  lB.v += lw[2] * w0 + lw[3] * q[2];
  lB.H += lw[3] * (q[0] + q[3]);
  lB.hq2 += lw[3] * q[1];
}

template <class real>
DFW_HD void unproject_adj(const Basis<real>& B, const real* q, const real* lw, real* lq, BasisAdj<real>& lB) {
  unproject_adj_B(B, q, lw, lB);
  unproject_adj_q(B, lw, lq);
}

template <class real>
DFW_HD void basis_adj_add(BasisAdj<real>& a, const BasisAdj<real>& b) {
  a.u += b.u;
  a.v += b.v;
  a.c += b.c;
  a.ic += b.ic;
  a.H += b.H;
  a.hq2 += b.hq2;
  a.b1 += b.b1;
  a.b2 += b.b2;
}

// Component C of project(B, w), and its adjoint (the four adjoints sum to project_adj).
template <int C, class real>
DFW_HD real project_comp(const Basis<real>& B, const real* w) {
  if (C == 2) return w[2] - B.v * w[0];
  const real T = B.b2 * w[0] - B.b1 * (B.u * w[1] + B.v * w[2] - w[3]);
  if (C == 1) return w[0] - T;
  const real s = (B.u * w[0] - w[1]) * B.ic;
  return C == 0 ? real(0.5) * (T + s) : real(0.5) * (T - s);
}

template <int C, class real>
DFW_HD void project_adj_comp(const Basis<real>& B, const real* w, real lqc, real* lw, BasisAdj<real>& lB) {
  if (C == 2) {
    lw[2] += lqc;
    lw[0] += -B.v * lqc;
    lB.v += -w[0] * lqc;
    return;
  }
  real lT, ls = real(0);
  if (C == 1) {
    lw[0] += lqc;
    lT = -lqc;
  } else {
    lT = real(0.5) * lqc;
    ls = C == 0 ? real(0.5) * lqc : real(-0.5) * lqc;
  }
  if (C != 1) {
    lB.u += ls * w[0] * B.ic;
    lw[0] += ls * B.u * B.ic;
    lw[1] += -ls * B.ic;
    lB.ic += ls * (B.u * w[0] - w[1]);
  }
  const real X = B.u * w[1] + B.v * w[2] - w[3];
  lB.b2 += lT * w[0];
  lw[0] += lT * B.b2;
  lB.b1 += -lT * X;
  const real lX = -lT * B.b1;
  lB.u += lX * w[1];
  lw[1] += lX * B.u;
  lB.v += lX * w[2];
  lw[2] += lX * B.v;
  lw[3] += -lX;
}

// Component C of R^T lw (the part of unproject_adj that does not depend on q).
template <int C, class real>
DFW_HD real unproject_adj_q_comp(const Basis<real>& B, const real* lw) {
  if (C == 2) return lw[2] + lw[3] * B.v;
  const real lw0 = lw[0] + B.u * lw[1] + B.v * lw[2];
  if (C == 1) return lw0 + lw[3] * B.hq2;
  const real ldq = B.c * lw[1] + B.u * B.c * lw[3];
  return C == 0 ? lw0 - ldq + lw[3] * B.H : lw0 + ldq + lw[3] * B.H;
}

// Basis part of unproject_adj for component C of q alone (the four parts sum to unproject_adj_B).
template <int C, class real>
DFW_HD void unproject_adj_B_comp(const Basis<real>& B, real qc, const real* lw, BasisAdj<real>& lB) {
  if (C == 0) {
    lB.u += lw[1] * qc - lw[3] * B.c * qc;
    lB.c += -lw[1] * qc - lw[3] * B.u * qc;
    lB.v += lw[2] * qc;
    lB.H += lw[3] * qc;
  } else if (C == 1) {
    lB.u += lw[1] * qc;
    lB.v += lw[2] * qc;
    lB.hq2 += lw[3] * qc;
  } else if (C == 2) {
    lB.v += lw[3] * qc;
  } else {
    lB.u += lw[1] * qc + lw[3] * B.c * qc;
    lB.c += lw[1] * qc + lw[3] * B.u * qc;
    lB.v += lw[2] * qc;
    lB.H += lw[3] * qc;
  }
}

// ------------------------------------------------------------------------------------------------
// Hybrid reconstruction: lP (NDEG coefficients) -> lQ (5) and the DF of the centre cell (DF branch).
// With a non-null P it also stores the forward polynomial (the same NDEG coefficients recon_poly
// gives, up to rounding: the reverse divides once per smoothness indicator and reuses the
// reciprocals).
// ------------------------------------------------------------------------------------------------
template <class real, int NDEG, int RULE = -1>
DFW_HD void recon_poly_adj(const real* Q, real a_lo, real a_c, real a_hi, const Coef<real>& k, const real* lP, real* lQ,
                           real& la_c, real* P = nullptr) {
  const real Q0 = Q[0], Q1 = Q[1], Q2 = Q[2], Q3 = Q[3], Q4 = Q[4];
  const real i6 = real(1.0 / 6.0);
  real p1_0 = (real(5) * Q2 + real(2) * Q3 - Q1) * i6;
  real p1_1 = Q3 - Q2;
  real p1_2 = real(0.5) * (Q1 + Q3) - Q2;
  real lP0 = lP[0], lP1 = NDEG > 1 ? lP[1] : real(0), lP2 = NDEG > 2 ? lP[2] : real(0);
  real lP3 = NDEG > 3 ? lP[3] : real(0), lP4 = NDEG > 4 ? lP[4] : real(0);
  real l10, l11, l12;  // adjoints of p1's coefficients
  if (df_switch<RULE>(a_lo, a_c, a_hi, k)) {
    la_c += lP0 * (p1_0 - Q2) + lP1 * p1_1 + lP2 * p1_2;
    lQ[2] += lP0 * (real(1) - a_c);
    if (P) {
      P[0] = Q2 + a_c * (p1_0 - Q2);
      if (NDEG > 1) P[1] = a_c * p1_1;
      if (NDEG > 2) P[2] = a_c * p1_2;
      if (NDEG > 3) P[3] = real(0);
      if (NDEG > 4) P[4] = real(0);
    }
    l10 = a_c * lP0;
    l11 = a_c * lP1;
    l12 = a_c * lP2;
  } else {
    real p0_0 = (real(2) * Q0 - real(7) * Q1 + real(11) * Q2) * i6;
    real p0_1 = Q0 - real(3) * Q1 + real(2) * Q2;
    real p0_2 = real(0.5) * (Q0 + Q2) - Q1;
    real p2_0 = (real(2) * Q2 + real(5) * Q3 - Q4) * i6;
    real p2_1 = Q3 - Q2;
    real p2_2 = real(0.5) * (Q2 + Q4) - Q3;
    real c0 = (real(2) * Q0 - real(13) * Q1 + real(47) * Q2 + real(27) * Q3 - real(3) * Q4) * real(1.0 / 60.0);
    real c1 = (Q1 - real(15) * Q2 + real(15) * Q3 - Q4) * real(1.0 / 12.0);
    real c2 = (-Q0 + real(6) * Q1 - real(8) * Q2 + real(2) * Q3 + Q4) * real(0.125);
    real c3 = (-Q1 + real(3) * Q2 - real(3) * Q3 + Q4) * i6;
    real c4 = (Q0 - real(4) * Q1 + real(6) * Q2 - real(4) * Q3 + Q4) * real(1.0 / 24.0);
    const real k1312 = real(13.0 / 12.0), k14 = real(0.25);
    real t0 = Q0 - real(2) * Q1 + Q2, s0 = Q0 - real(4) * Q1 + real(3) * Q2;
    real t1 = Q1 - real(2) * Q2 + Q3, s1 = Q1 - Q3;
    real t2 = Q2 - real(2) * Q3 + Q4, s2 = real(3) * Q2 - real(4) * Q3 + Q4;
    real b0 = k1312 * t0 * t0 + k14 * s0 * s0;
    real b1 = k1312 * t1 * t1 + k14 * s1 * s1;
    real b2 = k1312 * t2 * t2 + k14 * s2 * s2;
    real u1 = (real(11) * (Q0 - Q4) + real(82) * (Q3 - Q1)) * real(1.0 / 120.0);
    real u2 = (real(40) * (Q1 + Q3) - real(3) * (Q0 + Q4) - real(74) * Q2) * real(1.0 / 56.0);
    real u3 = (real(2) * (Q1 - Q3) + Q4 - Q0) * real(1.0 / 12.0);
    real u4 = c4;
    real e1 = u1 + real(0.1) * u3;
    real e2 = u2 + real(123.0 / 455.0) * u4;
    real b3 = e1 * e1 + real(13.0 / 3.0) * e2 * e2 + real(781.0 / 20.0) * u3 * u3 + real(1421461.0 / 2275.0) * u4 * u4;
    real tau = (fabs(b3 - b0) + fabs(b3 - b1) + fabs(b3 - b2)) * real(1.0 / 3.0);
    real be[4] = {b0 + k.eps, b1 + k.eps, b2 + k.eps, b3 + k.eps};
    const real i01 = rcp_pos(be[0] * be[1]), i23 = rcp_pos(be[2] * be[3]);
    real ib[4] = {be[1] * i01, be[0] * i01, be[3] * i23, be[2] * i23}, r[4], w[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      r[q] = tau * ib[q];
      w[q] = k.d[q] * (real(1) + r[q] * r[q]);
    }
    real iws = rcp_pos(w[0] + w[1] + w[2] + w[3]);
    real g3 = w[3] * iws;
    real g0 = w[0] * iws - g3 * k.dr[0];
    real g1 = w[1] * iws - g3 * k.dr[1];
    real g2 = w[2] * iws - g3 * k.dr[2];
    real h3 = g3 * k.inv_d3;
    if (P) {
      P[0] = g0 * p0_0 + g1 * p1_0 + g2 * p2_0 + h3 * c0;
      if (NDEG > 1) P[1] = g0 * p0_1 + g1 * p1_1 + g2 * p2_1 + h3 * c1;
      if (NDEG > 2) P[2] = g0 * p0_2 + g1 * p1_2 + g2 * p2_2 + h3 * c2;
      if (NDEG > 3) P[3] = h3 * c3;
      if (NDEG > 4) P[4] = h3 * c4;
    }
    // reverse of P
    real lg0 = lP0 * p0_0 + lP1 * p0_1 + lP2 * p0_2;
    real lg1 = lP0 * p1_0 + lP1 * p1_1 + lP2 * p1_2;
    real lg2 = lP0 * p2_0 + lP1 * p2_1 + lP2 * p2_2;
    real lh3 = lP0 * c0 + lP1 * c1 + lP2 * c2 + lP3 * c3 + lP4 * c4;
    real l00 = g0 * lP0, l01 = g0 * lP1, l02 = g0 * lP2;
    l10 = g1 * lP0;
    l11 = g1 * lP1;
    l12 = g1 * lP2;
    real l20 = g2 * lP0, l21 = g2 * lP1, l22 = g2 * lP2;
    real lc0 = h3 * lP0, lc1 = h3 * lP1, lc2 = h3 * lP2, lc3 = h3 * lP3, lc4 = h3 * lP4;
    // weights
    real lg3 = lh3 * k.inv_d3 - lg0 * k.dr[0] - lg1 * k.dr[1] - lg2 * k.dr[2];
    real lw[4] = {lg0 * iws, lg1 * iws, lg2 * iws, lg3 * iws};
    real liws = lg0 * w[0] + lg1 * w[1] + lg2 * w[2] + lg3 * w[3];
    real lS = -liws * iws * iws;
    real ltau = real(0), lb[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      lw[q] += lS;
      real lr = lw[q] * k.d[q] * real(2) * r[q] * ib[q];
      ltau += lr;
      lb[q] = -lr * r[q];
    }
    real s30 = sgn(b3 - b0), s31 = sgn(b3 - b1), s32 = sgn(b3 - b2);
    real lt3 = ltau * real(1.0 / 3.0);
    lb[3] += lt3 * (s30 + s31 + s32);
    lb[0] -= lt3 * s30;
    lb[1] -= lt3 * s31;
    lb[2] -= lt3 * s32;
    // b3
    real le1 = real(2) * e1 * lb[3];
    real le2 = real(26.0 / 3.0) * e2 * lb[3];
    real lu3 = real(781.0 / 10.0) * u3 * lb[3] + real(0.1) * le1;
    real lu4 = real(2.0 * 1421461.0 / 2275.0) * u4 * lb[3] + real(123.0 / 455.0) * le2;
    real lu1 = le1, lu2 = le2;
    lc4 += lu4;
    // u1..u3 -> Q
    lQ[0] += lu1 * real(11.0 / 120.0) - lu2 * real(3.0 / 56.0) - lu3 * real(1.0 / 12.0);
    lQ[1] += -lu1 * real(82.0 / 120.0) + lu2 * real(40.0 / 56.0) + lu3 * real(2.0 / 12.0);
    lQ[2] += -lu2 * real(74.0 / 56.0);
    lQ[3] += lu1 * real(82.0 / 120.0) + lu2 * real(40.0 / 56.0) - lu3 * real(2.0 / 12.0);
    lQ[4] += -lu1 * real(11.0 / 120.0) - lu2 * real(3.0 / 56.0) + lu3 * real(1.0 / 12.0);
    // b0..b2 -> Q
    real lt0 = real(2) * k1312 * t0 * lb[0], ls0 = real(2) * k14 * s0 * lb[0];
    real lt1 = real(2) * k1312 * t1 * lb[1], ls1 = real(2) * k14 * s1 * lb[1];
    real lt2 = real(2) * k1312 * t2 * lb[2], ls2 = real(2) * k14 * s2 * lb[2];
    lQ[0] += lt0 + ls0;
    lQ[1] += real(-2) * lt0 - real(4) * ls0 + lt1 + ls1;
    lQ[2] += lt0 + real(3) * ls0 - real(2) * lt1 + lt2 + real(3) * ls2;
    lQ[3] += lt1 - ls1 - real(2) * lt2 - real(4) * ls2;
    lQ[4] += lt2 + ls2;
    // candidates p0, p2 and the quartic -> Q
    lQ[0] += l00 * real(2.0 / 6.0) + l01 + real(0.5) * l02;
    lQ[1] += l00 * real(-7.0 / 6.0) - real(3) * l01 - l02;
    lQ[2] += l00 * real(11.0 / 6.0) + real(2) * l01 + real(0.5) * l02;
    lQ[2] += l20 * real(2.0 / 6.0) - l21 + real(0.5) * l22;
    lQ[3] += l20 * real(5.0 / 6.0) + l21 - l22;
    lQ[4] += l20 * real(-1.0 / 6.0) + real(0.5) * l22;
    lQ[0] += lc0 * real(2.0 / 60.0) - lc2 * real(0.125) + lc4 * real(1.0 / 24.0);
    lQ[1] += lc0 * real(-13.0 / 60.0) + lc1 * real(1.0 / 12.0) + lc2 * real(6.0 / 8.0) - lc3 * real(1.0 / 6.0) -
             lc4 * real(4.0 / 24.0);
    lQ[2] += lc0 * real(47.0 / 60.0) - lc1 * real(15.0 / 12.0) - lc2 + lc3 * real(3.0 / 6.0) + lc4 * real(6.0 / 24.0);
    lQ[3] += lc0 * real(27.0 / 60.0) + lc1 * real(15.0 / 12.0) + lc2 * real(2.0 / 8.0) - lc3 * real(3.0 / 6.0) -
             lc4 * real(4.0 / 24.0);
    lQ[4] += lc0 * real(-3.0 / 60.0) - lc1 * real(1.0 / 12.0) + lc2 * real(1.0 / 8.0) + lc3 * real(1.0 / 6.0) +
             lc4 * real(1.0 / 24.0);
  }
  // candidate p1 -> Q (both branches)
  lQ[1] += -l10 * i6 + real(0.5) * l12;
  lQ[2] += real(5) * l10 * i6 - l11 - l12;
  lQ[3] += real(2) * l10 * i6 + l11 + real(0.5) * l12;
}

// Reverse of recon_gauss: the adjoints lv, ld of the values and slopes at the two Gauss points ->
// lQ (5, accumulated) and the DF of the centre cell (DF branch).  Also returns the forward values
// and slopes (v, d), as recon_gauss computes them up to rounding.
template <class real, int RULE = -1>
DFW_HD void recon_gauss_adj(const real* Q, real a_lo, real a_c, real a_hi, const Coef<real>& k, const real* lv,
                            const real* ld, real* lQ, real& la_c, real* v, real* d) {
  const real Q1 = Q[1], Q2 = Q[2], Q3 = Q[3];
  const real dl = real(kGpDelta);
  // reverse of the even/odd split (linear, so it needs no forward value)
  const real lev = lv[0] + lv[1], lod = lv[1] - lv[0], levd = ld[0] + ld[1], lodd = ld[1] - ld[0];
  real lD1 = dl * lod + levd;
  real lD2 = real(2) * dl * lodd;
  real lD3 = dl * real(1.0 / 12.0) * lod + real(0.25) * levd;
  real lD4 = -real(1.0 / 180.0) * lev + dl * real(1.0 / 3.0) * lodd;
  lQ[2] += lev;
  real D1, D2, D3 = real(0), D4 = real(0);
  if (df_switch<RULE>(a_lo, a_c, a_hi, k)) {
    const real h1 = real(0.5) * (Q3 - Q1), h2 = real(0.5) * (Q1 - real(2) * Q2 + Q3);
    D1 = a_c * h1;
    D2 = a_c * h2;
    la_c += lD1 * h1 + lD2 * h2;
    const real m1 = real(0.5) * a_c * lD1, m2 = real(0.5) * a_c * lD2;
    lQ[1] += m2 - m1;
    lQ[2] -= real(2) * m2;
    lQ[3] += m1 + m2;
  } else {
    const WenoTerms<real> T = weno_terms(Q);
    const real b0 = T.b[0], b1 = T.b[1], b2 = T.b[2], b3 = T.b[3];
    const real tau = (fabs(b3 - b0) + fabs(b3 - b1) + fabs(b3 - b2)) * real(1.0 / 3.0);
    const real B0 = b0 + k.eps, B1 = b1 + k.eps, B2 = b2 + k.eps, B3 = b3 + k.eps;
    const real P01 = B0 * B1, P23 = B2 * B3, iP = rcp_pos(P01 * P23);
    const real a23 = P23 * iP, a01 = P01 * iP;
    const real ib[4] = {a23 * B1, a23 * B0, a01 * B3, a01 * B2};  // 1 / B_q
    real r[4], w[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      r[q] = tau * ib[q];
      w[q] = k.d[q] * (real(1) + r[q] * r[q]);
    }
    const real iws = rcp_pos(w[0] + w[1] + w[2] + w[3]);
    const real g3 = w[3] * iws;
    const real g0 = w[0] * iws - g3 * k.dr[0];
    const real g1 = w[1] * iws - g3 * k.dr[1];
    const real g2 = w[2] * iws - g3 * k.dr[2];
    const real h3 = g3 * k.inv_d3;
    const real q1 = T.u1 - real(0.15) * T.u3, q2 = T.u2 - real(3.0 / 14.0) * T.u4;
    D1 = real(0.5) * (g0 * T.s0 - g1 * T.s1 - g2 * T.s2) + h3 * q1;
    D2 = real(0.5) * (g0 * T.t0 + g1 * T.t1 + g2 * T.t2) + h3 * q2;
    D3 = h3 * T.u3;
    D4 = h3 * T.u4;
    // D1..D4 -> weights and terms
    const real lg0 = real(0.5) * (lD1 * T.s0 + lD2 * T.t0);
    const real lg1 = real(0.5) * (lD2 * T.t1 - lD1 * T.s1);
    const real lg2 = real(0.5) * (lD2 * T.t2 - lD1 * T.s2);
    const real lh3 = lD1 * q1 + lD2 * q2 + lD3 * T.u3 + lD4 * T.u4;
    real ls0 = real(0.5) * g0 * lD1, ls1 = -real(0.5) * g1 * lD1, ls2 = -real(0.5) * g2 * lD1;
    real lt0 = real(0.5) * g0 * lD2, lt1 = real(0.5) * g1 * lD2, lt2 = real(0.5) * g2 * lD2;
    real lu1 = h3 * lD1, lu2 = h3 * lD2;
    real lu3 = h3 * (lD3 - real(0.15) * lD1), lu4 = h3 * (lD4 - real(3.0 / 14.0) * lD2);
    // weights -> indicators
    const real lg3 = lh3 * k.inv_d3 - lg0 * k.dr[0] - lg1 * k.dr[1] - lg2 * k.dr[2];
    const real lgs[4] = {lg0, lg1, lg2, lg3};
    const real lS = -(lg0 * w[0] + lg1 * w[1] + lg2 * w[2] + lg3 * w[3]) * iws * iws;
    real ltau = real(0), lb[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const real lr = (lgs[q] * iws + lS) * k.d[q] * real(2) * r[q];
      ltau += lr * ib[q];
      lb[q] = -lr * r[q] * ib[q];
    }
    const real s30 = sgn(b3 - b0), s31 = sgn(b3 - b1), s32 = sgn(b3 - b2);
    const real lt3 = ltau * real(1.0 / 3.0);
    lb[3] += lt3 * (s30 + s31 + s32);
    lb[0] -= lt3 * s30;
    lb[1] -= lt3 * s31;
    lb[2] -= lt3 * s32;
    // indicators -> terms
    const real k1312 = real(13.0 / 12.0), k14 = real(0.25);
    lt0 += real(2) * k1312 * T.t0 * lb[0];
    ls0 += real(2) * k14 * T.s0 * lb[0];
    lt1 += real(2) * k1312 * T.t1 * lb[1];
    ls1 += real(2) * k14 * T.s1 * lb[1];
    lt2 += real(2) * k1312 * T.t2 * lb[2];
    ls2 += real(2) * k14 * T.s2 * lb[2];
    const real e1 = T.u1 + real(0.1) * T.u3, e2 = T.u2 + real(123.0 / 455.0) * T.u4;
    const real le1 = real(2) * e1 * lb[3], le2 = real(26.0 / 3.0) * e2 * lb[3];
    lu1 += le1;
    lu2 += le2;
    lu3 += real(781.0 / 10.0) * T.u3 * lb[3] + real(0.1) * le1;
    lu4 += real(2.0 * 1421461.0 / 2275.0) * T.u4 * lb[3] + real(123.0 / 455.0) * le2;
    // terms -> averages: u1 = (-11 d40 - 82 s1)/120, u2 = (34 t1 - 3 (t0 + t2))/56,
    // u3 = (2 s1 + d40)/12, u4 = (t0 - 2 t1 + t2)/24, d40 = Q4 - Q0, s2 = t2 - 2 (Q3 - Q2)
    const real ld40 = -real(11.0 / 120.0) * lu1 + real(1.0 / 12.0) * lu3;
    ls1 += -real(82.0 / 120.0) * lu1 + real(2.0 / 12.0) * lu3;
    lt1 += real(34.0 / 56.0) * lu2 - real(2.0 / 24.0) * lu4;
    lt0 += -real(3.0 / 56.0) * lu2 + real(1.0 / 24.0) * lu4;
    lt2 += -real(3.0 / 56.0) * lu2 + real(1.0 / 24.0) * lu4 + ls2;
    lQ[0] += lt0 + ls0 - ld40;
    lQ[1] += -real(2) * lt0 + lt1 - real(4) * ls0 + ls1;
    lQ[2] += lt0 - real(2) * lt1 + lt2 + real(3) * ls0 + real(2) * ls2;
    lQ[3] += lt1 - real(2) * lt2 - ls1 - real(2) * ls2;
    lQ[4] += lt2 + ld40;
  }
  const real ev = Q2 - real(1.0 / 180.0) * D4, od = dl * (D1 + real(1.0 / 12.0) * D3);
  const real evd = D1 + real(0.25) * D3, odd = dl * (real(2) * D2 + real(1.0 / 3.0) * D4);
  v[0] = ev - od;
  v[1] = ev + od;
  d[0] = evd - odd;
  d[1] = evd + odd;
}

// ------------------------------------------------------------------------------------------------
// Primitive variables and the DF of one Gauss point.
// ------------------------------------------------------------------------------------------------
template <class real>
struct PrimAdj {
  real r, ir, u, v, p, c;
  DFW_HD void zero() { r = ir = u = v = p = c = real(0); }
};

template <class real>
DFW_HD void prim_adj(const real* w, const Prim<real>& q, const Coef<real>& k, const PrimAdj<real>& lq, real* lw) {
  real l_p = lq.p + lq.c * k.gamma * q.ir * real(0.5) / q.c;
  real l_ir = lq.ir + lq.c * k.gamma * q.p * real(0.5) / q.c;
  real l_u = lq.u - real(0.5) * k.gm1 * w[1] * l_p;
  real l_v = lq.v - real(0.5) * k.gm1 * w[2] * l_p;
  lw[3] += k.gm1 * l_p;
  lw[1] += -real(0.5) * k.gm1 * q.u * l_p + l_u * q.ir;
  lw[2] += -real(0.5) * k.gm1 * q.v * l_p + l_v * q.ir;
  l_ir += l_u * w[1] + l_v * w[2];
  lw[0] += lq.r - l_ir * q.ir * q.ir;
}

template <class real>
DFW_HD void df_factor_adj(const Prim<real>& L, const Prim<real>& R, real lalpha, PrimAdj<real>& lL, PrimAdj<real>& lR) {
  real jump = fabs(L.p - R.p);
  real icl = real(1) / L.c, icr = real(1) / R.c;
  real dn = L.u * icl - R.u * icr;
  real dt = L.v * icl - R.v * icr;
  real D = jump * (real(1) / L.p + real(1) / R.p) + dn * dn + dt * dt;
  real a = real(1) / (real(1) + D * D);
  real lD = -real(2) * D * a * a * lalpha;
  real ljump = lD * (real(1) / L.p + real(1) / R.p);
  lL.p += -lD * jump / (L.p * L.p);
  lR.p += -lD * jump / (R.p * R.p);
  real s = sgn(L.p - R.p);
  lL.p += s * ljump;
  lR.p -= s * ljump;
  real ldn = real(2) * dn * lD, ldt = real(2) * dt * lD;
  lL.u += ldn * icl;
  lR.u -= ldn * icr;
  lL.v += ldt * icl;
  lR.v -= ldt * icr;
  real licl = ldn * L.u + ldt * L.v;
  real licr = -(ldn * R.u + ldt * R.v);
  lL.c += -licl * icl * icl;
  lR.c += -licr * icr * icr;
}

// ------------------------------------------------------------------------------------------------
// Lax-Friedrichs flux with the Cauchy-Kovalevskaya time derivative.
// ------------------------------------------------------------------------------------------------
template <class real>
DFW_HD void euler_time_derivs_adj(const real* w, const Prim<real>& q, const real* wx, const real* wy,
                                  const Coef<real>& k, const real* lwt_in, const real* lft, real* lw, PrimAdj<real>& lq,
                                  real* lwx, real* lwy) {
  // forward
  real ke = real(0.5) * (q.u * q.u + q.v * q.v);
  real ux = (wx[1] - q.u * wx[0]) * q.ir, vx = (wx[2] - q.v * wx[0]) * q.ir;
  real px = k.gm1 * (wx[3] - q.u * wx[1] - q.v * wx[2] + ke * wx[0]);
  real uy = (wy[1] - q.u * wy[0]) * q.ir, vy = (wy[2] - q.v * wy[0]) * q.ir;
  real py = k.gm1 * (wy[3] - q.u * wy[1] - q.v * wy[2] + ke * wy[0]);
  real rt = -(q.u * wx[0] + q.r * ux + q.v * wy[0] + q.r * vy);
  real ut = -(q.u * ux + q.v * uy + px * q.ir);
  real vt = -(q.u * vx + q.v * vy + py * q.ir);
  real pt = -(q.u * px + q.v * py + k.gamma * q.p * (ux + vy));
  real wt1 = rt * q.u + q.r * ut;
  real wt3 = pt * k.inv_gm1 + rt * ke + q.r * (q.u * ut + q.v * vt);
  // reverse
  real lwt[4] = {lwt_in[0], lwt_in[1], lwt_in[2], lwt_in[3]};
  real lut = real(0), lvt = real(0), lpt = real(0), lrt = real(0), lke = real(0);
  // ft3 = ut (w3 + p) + u (wt3 + pt)
  lut += lft[3] * (w[3] + q.p);
  lw[3] += lft[3] * ut;
  lq.p += lft[3] * ut;
  lq.u += lft[3] * (wt3 + pt);
  lwt[3] += lft[3] * q.u;
  lpt += lft[3] * q.u;
  // ft2 = wt1 v + w1 vt
  lwt[1] += lft[2] * q.v;
  lq.v += lft[2] * wt1;
  lw[1] += lft[2] * vt;
  lvt += lft[2] * w[1];
  // ft1 = wt1 u + w1 ut + pt
  lwt[1] += lft[1] * q.u;
  lq.u += lft[1] * wt1;
  lw[1] += lft[1] * ut;
  lut += lft[1] * w[1];
  lpt += lft[1];
  // ft0 = wt1
  lwt[1] += lft[0];
  // wt3 = pt/gm1 + rt ke + r (u ut + v vt)
  lpt += lwt[3] * k.inv_gm1;
  lrt += lwt[3] * ke;
  lke += lwt[3] * rt;
  lq.r += lwt[3] * (q.u * ut + q.v * vt);
  lq.u += lwt[3] * q.r * ut;
  lut += lwt[3] * q.r * q.u;
  lq.v += lwt[3] * q.r * vt;
  lvt += lwt[3] * q.r * q.v;
  // wt2 = rt v + r vt
  lrt += lwt[2] * q.v;
  lq.v += lwt[2] * rt;
  lq.r += lwt[2] * vt;
  lvt += lwt[2] * q.r;
  // wt1 = rt u + r ut
  lrt += lwt[1] * q.u;
  lq.u += lwt[1] * rt;
  lq.r += lwt[1] * ut;
  lut += lwt[1] * q.r;
  // wt0 = rt
  lrt += lwt[0];
  // pt = -(u px + v py + gamma p (ux + vy))
  real lux = -lpt * k.gamma * q.p, lvy = -lpt * k.gamma * q.p;
  real lpx = -lpt * q.u, lpy = -lpt * q.v;
  lq.u += -lpt * px;
  lq.v += -lpt * py;
  lq.p += -lpt * k.gamma * (ux + vy);
  // vt = -(u vx + v vy + py ir)
  lq.u -= lvt * vx;
  real lvx = -lvt * q.u;
  lq.v -= lvt * vy;
  lvy -= lvt * q.v;
  lpy -= lvt * q.ir;
  lq.ir -= lvt * py;
  // ut = -(u ux + v uy + px ir)
  lq.u -= lut * ux;
  lux -= lut * q.u;
  lq.v -= lut * uy;
  real luy = -lut * q.v;
  lpx -= lut * q.ir;
  lq.ir -= lut * px;
  // rt = -(u wx0 + r ux + v wy0 + r vy)
  lq.u -= lrt * wx[0];
  lwx[0] -= lrt * q.u;
  lq.r -= lrt * (ux + vy);
  lux -= lrt * q.r;
  lq.v -= lrt * wy[0];
  lwy[0] -= lrt * q.v;
  lvy -= lrt * q.r;
  // py, px
  lwy[3] += k.gm1 * lpy;
  lq.u -= k.gm1 * lpy * wy[1];
  lwy[1] -= k.gm1 * lpy * q.u;
  lq.v -= k.gm1 * lpy * wy[2];
  lwy[2] -= k.gm1 * lpy * q.v;
  lke += k.gm1 * lpy * wy[0];
  lwy[0] += k.gm1 * lpy * ke;
  lwx[3] += k.gm1 * lpx;
  lq.u -= k.gm1 * lpx * wx[1];
  lwx[1] -= k.gm1 * lpx * q.u;
  lq.v -= k.gm1 * lpx * wx[2];
  lwx[2] -= k.gm1 * lpx * q.v;
  lke += k.gm1 * lpx * wx[0];
  lwx[0] += k.gm1 * lpx * ke;
  // vy, uy, vx, ux
  lwy[2] += lvy * q.ir;
  lq.v -= lvy * wy[0] * q.ir;
  lwy[0] -= lvy * q.v * q.ir;
  lq.ir += lvy * (wy[2] - q.v * wy[0]);
  lwy[1] += luy * q.ir;
  lq.u -= luy * wy[0] * q.ir;
  lwy[0] -= luy * q.u * q.ir;
  lq.ir += luy * (wy[1] - q.u * wy[0]);
  lwx[2] += lvx * q.ir;
  lq.v -= lvx * wx[0] * q.ir;
  lwx[0] -= lvx * q.v * q.ir;
  lq.ir += lvx * (wx[2] - q.v * wx[0]);
  lwx[1] += lux * q.ir;
  lq.u -= lux * wx[0] * q.ir;
  lwx[0] -= lux * q.u * q.ir;
  lq.ir += lux * (wx[1] - q.u * wx[0]);
  // ke
  lq.u += lke * q.u;
  lq.v += lke * q.v;
}

template <class real>
DFW_HD void lf_flux_adj(const real* wl, const real* wlx, const real* wly, const real* wr, const real* wrx,
                        const real* wry, const Prim<real>& ql, const Prim<real>& qr, const Coef<real>& k,
                        const real* lF, const real* lFt, real* lwl, real* lwlx, real* lwly, real* lwr, real* lwrx,
                        real* lwry, PrimAdj<real>& lql, PrimAdj<real>& lqr) {
  real sl = fabs(ql.u) + ql.c, sr = fabs(qr.u) + qr.c;
  const bool left = sl >= sr;
  real s = left ? sl : sr;
  real hs = real(0.5) * s;
  real wtl[4], ftl[4], wtr[4], ftr[4];
  euler_time_derivs(wl, ql, wlx, wly, k, wtl, ftl);
  euler_time_derivs(wr, qr, wrx, wry, k, wtr, ftr);
  real lhs = real(0);
  real lwtl[4], lwtr[4], lftl[4], lftr[4];
  real lFl[4], lFr[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    lhs -= lF[c] * (wr[c] - wl[c]) + lFt[c] * (wtr[c] - wtl[c]);
    lwr[c] -= hs * lF[c];
    lwl[c] += hs * lF[c];
    lFl[c] = real(0.5) * lF[c];
    lFr[c] = real(0.5) * lF[c];
    lwtr[c] = -hs * lFt[c];
    lwtl[c] = hs * lFt[c];
    lftl[c] = real(0.5) * lFt[c];
    lftr[c] = real(0.5) * lFt[c];
  }
  real ls = real(0.5) * lhs;
  if (left) {
    lql.u += sgn(ql.u) * ls;
    lql.c += ls;
  } else {
    lqr.u += sgn(qr.u) * ls;
    lqr.c += ls;
  }
  // F = (w1, w1 u + p, w2 u, u (w3 + p)) on each side
  lwl[1] += lFl[0] + lFl[1] * ql.u;
  lql.u += lFl[1] * wl[1] + lFl[2] * wl[2] + lFl[3] * (wl[3] + ql.p);
  lql.p += lFl[1] + lFl[3] * ql.u;
  lwl[2] += lFl[2] * ql.u;
  lwl[3] += lFl[3] * ql.u;
  lwr[1] += lFr[0] + lFr[1] * qr.u;
  lqr.u += lFr[1] * wr[1] + lFr[2] * wr[2] + lFr[3] * (wr[3] + qr.p);
  lqr.p += lFr[1] + lFr[3] * qr.u;
  lwr[2] += lFr[2] * qr.u;
  lwr[3] += lFr[3] * qr.u;
  euler_time_derivs_adj(wl, ql, wlx, wly, k, lwtl, lftl, lwl, lql, lwlx, lwly);
  euler_time_derivs_adj(wr, qr, wrx, wry, k, lwtr, lftr, lwr, lqr, lwrx, lwry);
}

// ------------------------------------------------------------------------------------------------
// Gas-kinetic flux.
// ------------------------------------------------------------------------------------------------
template <class real>
struct MomAdj {
  real mu[7], mv[6], mx[3];
  DFW_HD void zero() {
#pragma unroll
    for (int i = 0; i < 7; ++i) mu[i] = real(0);
#pragma unroll
    for (int i = 0; i < 6; ++i) mv[i] = real(0);
#pragma unroll
    for (int i = 0; i < 3; ++i) mx[i] = real(0);
  }
};

template <class real>
DFW_HD void mom_adj(const Mom<real>& M, int a, int b, int c, real l, MomAdj<real>& lM) {
  lM.mu[a] += l * M.mv[b] * M.mx[c];
  lM.mv[b] += l * M.mu[a] * M.mx[c];
  lM.mx[c] += l * M.mu[a] * M.mv[b];
}

// <(s.psi) u^a v^b xi^2c>: adjoint into the slope and the moments
template <class real>
DFW_HD void mom_s_adj(const Mom<real>& M, const real* s, int a, int b, int c, real l, real* ls, MomAdj<real>& lM) {
  ls[0] += l * mom(M, a, b, c);
  ls[1] += l * mom(M, a + 1, b, c);
  ls[2] += l * mom(M, a, b + 1, c);
  ls[3] += l * real(0.5) * (mom(M, a + 2, b, c) + mom(M, a, b + 2, c) + mom(M, a, b, c + 1));
  mom_adj(M, a, b, c, l * s[0], lM);
  mom_adj(M, a + 1, b, c, l * s[1], lM);
  mom_adj(M, a, b + 1, c, l * s[2], lM);
  const real h3 = real(0.5) * s[3] * l;
  mom_adj(M, a + 2, b, c, h3, lM);
  mom_adj(M, a, b + 2, c, h3, lM);
  mom_adj(M, a, b, c + 1, h3, lM);
}

template <class real>
DFW_HD void mom_s_psi_adj(const Mom<real>& M, const real* s, int a, int b, const real* l, real* ls, MomAdj<real>& lM) {
  mom_s_adj(M, s, a, b, 0, l[0], ls, lM);
  mom_s_adj(M, s, a + 1, b, 0, l[1], ls, lM);
  mom_s_adj(M, s, a, b + 1, 0, l[2], ls, lM);
  const real h = real(0.5) * l[3];
  mom_s_adj(M, s, a + 2, b, 0, h, ls, lM);
  mom_s_adj(M, s, a, b + 2, 0, h, ls, lM);
  mom_s_adj(M, s, a, b, 1, h, ls, lM);
}

template <class real>
DFW_HD void mom_psi_adj(const Mom<real>& M, int a, int b, const real* l, MomAdj<real>& lM) {
  mom_adj(M, a, b, 0, l[0], lM);
  mom_adj(M, a + 1, b, 0, l[1], lM);
  mom_adj(M, a, b + 1, 0, l[2], lM);
  const real h = real(0.5) * l[3];
  mom_adj(M, a + 2, b, 0, h, lM);
  mom_adj(M, a, b + 2, 0, h, lM);
  mom_adj(M, a, b, 1, h, lM);
}

// Reverse of maxwell_moments: -> adjoints of U, V, lambda.
template <class real>
DFW_HD void maxwell_moments_adj(const Mom<real>& M, int side, const Coef<real>& k, MomAdj<real> lM, real& lU, real& lV,
                                real& llam) {
  const real U = M.U, V = M.V, lam = M.lam;
  const real h = real(0.5) / lam;
  real lh = lM.mx[1] * k.K + lM.mx[2] * real(2) * k.K * (k.K + real(2)) * h;
#pragma unroll
  for (int n = 3; n >= 0; --n) {  // mv[n+2] = V mv[n+1] + (n+1) h mv[n]
    const real l = lM.mv[n + 2];
    lV += l * M.mv[n + 1];
    lM.mv[n + 1] += l * V;
    lh += l * real(n + 1) * M.mv[n];
    lM.mv[n] += l * real(n + 1) * h;
  }
  lV += lM.mv[1];
#pragma unroll
  for (int n = 4; n >= 0; --n) {
    const real l = lM.mu[n + 2];
    lU += l * M.mu[n + 1];
    lM.mu[n + 1] += l * U;
    lh += l * real(n + 1) * M.mu[n];
    lM.mu[n] += l * real(n + 1) * h;
  }
  if (side == 0) {
    lU += lM.mu[1];
  } else {
    const real inv_sqrt_pi = real(0.56418958354775628695);
    const real sg = side > 0 ? real(1) : real(-1);
    real sl = sqrt(lam);
    real ex = exp(-lam * U * U);
    real g = real(0.5) * ex * inv_sqrt_pi / sl;
    // mu1 = U mu0 +- g
    lU += lM.mu[1] * M.mu[0];
    real lmu0 = lM.mu[0] + lM.mu[1] * U;
    real lg = sg * lM.mu[1];
    // mu0 = erfc(-sg sl U)/2: d/dz erfc(z)/2 = -exp(-z^2)/sqrt(pi), z = -sg sl U
    real dmu0 = -inv_sqrt_pi * ex;
    lU += lmu0 * dmu0 * (-sg * sl);
    real lsl = lmu0 * dmu0 * (-sg * U);
    // g = exp(-lam U^2) / (2 sqrt(pi) sl)
    lU += lg * g * (real(-2) * lam * U);
    llam += lg * g * (-U * U);
    lsl += -lg * g / sl;
    llam += lsl * real(0.5) / sl;
  }
  llam += -lh * real(0.5) / (lam * lam);
}

template <class real>
DFW_HD void micro_slope_adj(const real* g, real U, real V, real lam, const Coef<real>& k, const real* ls_in, real* lg,
                            real& lU, real& lV, real& llam) {
  const real K2 = k.K2;
  const real ilam = real(1) / lam;
  real B = U * U + V * V + K2 * real(0.5) * ilam;
  real R4 = real(2) * g[3] - B * g[0];
  real R3 = g[2] - V * g[0];
  real R2 = g[1] - U * g[0];
  real kap = k.k4K2 * (lam * lam);
  real Z = R4 - real(2) * U * R2 - real(2) * V * R3;
  real s3 = kap * Z;
  real s2 = real(2) * lam * R3 - V * s3;
  real s1 = real(2) * lam * R2 - U * s3;
  // s0 = g0 - U s1 - V s2 - s3 B / 2
  real ls1 = ls_in[1] - U * ls_in[0];
  real ls2 = ls_in[2] - V * ls_in[0];
  real ls3 = ls_in[3] - real(0.5) * B * ls_in[0];
  lg[0] += ls_in[0];
  lU -= ls_in[0] * s1;
  lV -= ls_in[0] * s2;
  real lB = -real(0.5) * s3 * ls_in[0];
  // s1 = 2 lam R2 - U s3 ; s2 = 2 lam R3 - V s3
  llam += real(2) * R2 * ls1 + real(2) * R3 * ls2;
  real lR2 = real(2) * lam * ls1, lR3 = real(2) * lam * ls2;
  lU -= s3 * ls1;
  lV -= s3 * ls2;
  ls3 -= U * ls1 + V * ls2;
  // s3 = kap Z
  llam += ls3 * Z * real(2) * lam * k.k4K2;
  real lZ = ls3 * kap;
  real lR4 = lZ;
  lU -= real(2) * R2 * lZ;
  lR2 -= real(2) * U * lZ;
  lV -= real(2) * R3 * lZ;
  lR3 -= real(2) * V * lZ;
  lg[1] += lR2;
  lU -= g[0] * lR2;
  lg[0] -= U * lR2;
  lg[2] += lR3;
  lV -= g[0] * lR3;
  lg[0] -= V * lR3;
  lg[3] += real(2) * lR4;
  lB -= g[0] * lR4;
  lg[0] -= B * lR4;
  lU += real(2) * U * lB;
  lV += real(2) * V * lB;
  llam += -K2 * real(0.5) * (ilam * ilam) * lB;
}

// Adjoint of gks_flux (lF may be null when the flux itself was not requested), in two halves.  The first recomputes the flux and reverses its time
// coefficients and the equilibrium-state part, down to the adjoints of the half-space sums
// (Wc, Wcn, Wct, Flr, Malr) and the pressure-jump term of tau; the second reverses the two
// half-space sides.  A caller short of registers can keep the handover in memory between them;
// gks_flux_adj runs both in turn.
template <class real>
struct GksEqAdj {
  real lWc[4], lWcn[4], lWct[4], lFlr[4], lMalr[4];
  real lpl, lpr;  // the tau term's adjoints of the left and right pressure
};

template <class real>
DFW_HD void gks_flux_adj_eq(const real* wln, const real* wlt, const real* wrn, const real* wrt, const Prim<real>& ql,
                            const Prim<real>& qr, real dt, const Coef<real>& k, const real* lF, const real* lFt,
                            GksEqAdj<real>& e) {
  // ---- forward recompute
  real Wc[4] = {0, 0, 0, 0}, Wcn[4] = {0, 0, 0, 0}, Wct[4] = {0, 0, 0, 0};
  real Flr[4] = {0, 0, 0, 0}, Malr[4] = {0, 0, 0, 0};
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const real* wn = side == 0 ? wln : wrn;
    const real* wt = side == 0 ? wlt : wrt;
    const Prim<real>& q = side == 0 ? ql : qr;
    real lam = real(0.5) * q.r / q.p;
    Mom<real> M;
    maxwell_moments(q.u, q.v, lam, side == 0 ? 1 : -1, k, M);
    real g[4], a[4], b[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) g[c] = wn[c] * q.ir;
    micro_slope(g, q.u, q.v, lam, real(0.5) / lam, k, a);
#pragma unroll
    for (int c = 0; c < 4; ++c) g[c] = wt[c] * q.ir;
    micro_slope(g, q.u, q.v, lam, real(0.5) / lam, k, b);
    real t0[4], t1[4], t2[4];
    mom_psi(M, 0, 0, t0);
    mom_s_psi(M, a, 0, 0, t1);
    mom_s_psi(M, b, 0, 0, t2);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      Wc[c] += q.r * t0[c];
      Wcn[c] += q.r * t1[c];
      Wct[c] += q.r * t2[c];
    }
    mom_psi(M, 1, 0, t0);
    mom_s_psi(M, a, 2, 0, t1);
    mom_s_psi(M, b, 1, 1, t2);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      Flr[c] += q.r * t0[c];
      Malr[c] += q.r * (t1[c] + t2[c]);
    }
  }
  real irc = real(1) / Wc[0];
  real Uc = Wc[1] * irc, Vc = Wc[2] * irc;
  real pc = k.gm1 * (Wc[3] - real(0.5) * (Wc[1] * Uc + Wc[2] * Vc));
  real lamc = real(0.5) * Wc[0] / pc;
  Mom<real> Mc;
  maxwell_moments(Uc, Vc, lamc, 0, k, Mc);
  real gn[4], gt[4], ac[4], bc[4], Ac[4], gA[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    gn[c] = Wcn[c] * irc;
    gt[c] = Wct[c] * irc;
  }
  micro_slope(gn, Uc, Vc, lamc, real(0.5) / lamc, k, ac);
  micro_slope(gt, Uc, Vc, lamc, real(0.5) / lamc, k, bc);
  real y1[4], y2[4];
  mom_s_psi(Mc, ac, 1, 0, y1);
  mom_s_psi(Mc, bc, 0, 1, y2);
#pragma unroll
  for (int c = 0; c < 4; ++c) gA[c] = -(y1[c] + y2[c]);
  micro_slope(gA, Uc, Vc, lamc, real(0.5) / lamc, k, Ac);
  real fc[4], x1[4], x2[4], xA[4];
  mom_psi(Mc, 1, 0, fc);
  mom_s_psi(Mc, ac, 2, 0, x1);
  mom_s_psi(Mc, bc, 1, 1, x2);
  mom_s_psi(Mc, Ac, 1, 0, xA);
  real Fc[4], Mac[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    Fc[c] = Wc[0] * fc[c];
    Mac[c] = Wc[0] * (x1[c] + x2[c]);
  }
  const real pq = (ql.p - qr.p) / (ql.p + qr.p);
  real tau = k.c1 * dt + k.c2 * fabs(pq) * dt;
  real E2 = exp(-real(0.5) * dt / tau);
  real E1 = E2 * E2;
  real om = real(1) - E2;
  real idt = real(1) / dt;
  real ct1 = real(4) * tau * om * om * idt * idt;
  real ct2 = real(4) * (tau * dt * E2 * om - tau * tau * om * om) * idt * idt;
  real z = real(3) - real(4) * E2 + E1;
  real cf1 = real(1) - tau * idt * z;
  real cf2 = tau * tau * idt * z + tau * (E1 - real(2) * E2);
  // ---- reverse: time coefficients
  real lFc[4], lMac[4], lMAc[4];
  real* lFlr = e.lFlr;
  real* lMalr = e.lMalr;
  e.lpl = e.lpr = real(0);
  real lct1 = real(0), lct2 = real(0), lcf1 = real(0), lcf2 = real(0);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const real MA = Wc[0] * xA[c];
    (void)MA;
    lct1 += lFt[c] * (Fc[c] - Flr[c]);
    lct2 += lFt[c] * (Mac[c] - Malr[c]);
    lFc[c] = ct1 * lFt[c];
    lFlr[c] = -ct1 * lFt[c];
    lMac[c] = ct2 * lFt[c];
    lMalr[c] = -ct2 * lFt[c];
    lMAc[c] = lFt[c];
    if (lF) {
      lcf1 += lF[c] * (Fc[c] - Flr[c]);
      lcf2 += lF[c] * (Mac[c] - Malr[c]);
      lFc[c] += cf1 * lF[c];
      lFlr[c] += (real(1) - cf1) * lF[c];
      lMac[c] += cf2 * lF[c];
      lMalr[c] -= cf2 * lF[c];
    }
  }
  if (tau > real(0)) {
    real dE2 = E2 * real(0.5) * dt / (tau * tau);
    real dct1 = real(4) * idt * idt * (om * om - real(2) * tau * om * dE2);
    real dct2 = real(4) * idt * idt *
                (dt * E2 * om + tau * dt * (dE2 * om - E2 * dE2) - real(2) * tau * om * om + real(2) * tau * tau * om * dE2);
    real dz = (real(-4) + real(2) * E2) * dE2;
    real dcf1 = -idt * (z + tau * dz);
    real dcf2 = real(2) * tau * idt * z + tau * tau * idt * dz + (E1 - real(2) * E2) + tau * (real(2) * E2 - real(2)) * dE2;
    real ltau = lct1 * dct1 + lct2 * dct2 + lcf1 * dcf1 + lcf2 * dcf2;
    real lpq = ltau * k.c2 * dt * sgn(pq);
    real isum = real(1) / (ql.p + qr.p);
    e.lpl = lpq * (real(1) - pq) * isum;
    e.lpr = lpq * (real(-1) - pq) * isum;
  }
  // ---- reverse: equilibrium-state fluxes
  MomAdj<real> lMc;
  lMc.zero();
  real* lWc = e.lWc;
  real* lWcn = e.lWcn;
  real* lWct = e.lWct;
#pragma unroll
  for (int c = 0; c < 4; ++c) lWc[c] = lWcn[c] = lWct[c] = real(0);
  real lac[4] = {0, 0, 0, 0}, lbc[4] = {0, 0, 0, 0}, lAc[4] = {0, 0, 0, 0};
  real lx[4], lfc[4], lxA[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    lWc[0] += lFc[c] * fc[c] + lMac[c] * (x1[c] + x2[c]) + lMAc[c] * xA[c];
    lfc[c] = Wc[0] * lFc[c];
    lx[c] = Wc[0] * lMac[c];
    lxA[c] = Wc[0] * lMAc[c];
  }
  mom_psi_adj(Mc, 1, 0, lfc, lMc);
  mom_s_psi_adj(Mc, ac, 2, 0, lx, lac, lMc);
  mom_s_psi_adj(Mc, bc, 1, 1, lx, lbc, lMc);
  mom_s_psi_adj(Mc, Ac, 1, 0, lxA, lAc, lMc);
  real lUc = real(0), lVc = real(0), llamc = real(0);
  real lgA[4] = {0, 0, 0, 0};
  micro_slope_adj(gA, Uc, Vc, lamc, k, lAc, lgA, lUc, lVc, llamc);
  real ly[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) ly[c] = -lgA[c];
  mom_s_psi_adj(Mc, ac, 1, 0, ly, lac, lMc);
  mom_s_psi_adj(Mc, bc, 0, 1, ly, lbc, lMc);
  real lgn[4] = {0, 0, 0, 0}, lgt[4] = {0, 0, 0, 0};
  micro_slope_adj(gn, Uc, Vc, lamc, k, lac, lgn, lUc, lVc, llamc);
  micro_slope_adj(gt, Uc, Vc, lamc, k, lbc, lgt, lUc, lVc, llamc);
  real lirc = real(0);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    lWcn[c] += lgn[c] * irc;
    lWct[c] += lgt[c] * irc;
    lirc += lgn[c] * Wcn[c] + lgt[c] * Wct[c];
  }
  maxwell_moments_adj(Mc, 0, k, lMc, lUc, lVc, llamc);
  // lamc = Wc0 / (2 pc), pc = gm1 (Wc3 - (Wc1 Uc + Wc2 Vc)/2), Uc = Wc1 irc, Vc = Wc2 irc, irc = 1/Wc0
  lWc[0] += llamc * real(0.5) / pc;
  real lpc = -llamc * lamc / pc;
  lWc[3] += lpc * k.gm1;
  lWc[1] += -lpc * k.gm1 * real(0.5) * Uc;
  lWc[2] += -lpc * k.gm1 * real(0.5) * Vc;
  lUc += -lpc * k.gm1 * real(0.5) * Wc[1];
  lVc += -lpc * k.gm1 * real(0.5) * Wc[2];
  lWc[1] += lUc * irc;
  lWc[2] += lVc * irc;
  lirc += lUc * Wc[1] + lVc * Wc[2];
  lWc[0] += -lirc * irc * irc;
}

template <class real>
DFW_HD void gks_flux_adj_sides(const real* wln, const real* wlt, const real* wrn, const real* wrt,
                               const Prim<real>& ql, const Prim<real>& qr, const Coef<real>& k,
                               const GksEqAdj<real>& e, real* lwln, real* lwlt, real* lwrn, real* lwrt,
                               PrimAdj<real>& lql, PrimAdj<real>& lqr) {
  const real* lWc = e.lWc;
  const real* lWcn = e.lWcn;
  const real* lWct = e.lWct;
  const real* lFlr = e.lFlr;
  const real* lMalr = e.lMalr;
  lql.p += e.lpl;
  lqr.p += e.lpr;
  // ---- reverse: the two half-space sides
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const real* wn = side == 0 ? wln : wrn;
    const real* wt = side == 0 ? wlt : wrt;
    real* lwn = side == 0 ? lwln : lwrn;
    real* lwt = side == 0 ? lwlt : lwrt;
    const Prim<real>& q = side == 0 ? ql : qr;
    PrimAdj<real>& lq = side == 0 ? lql : lqr;
    real lam = real(0.5) * q.r / q.p;
    Mom<real> M;
    maxwell_moments(q.u, q.v, lam, side == 0 ? 1 : -1, k, M);
    real g1[4], g2[4], a[4], b[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      g1[c] = wn[c] * q.ir;
      g2[c] = wt[c] * q.ir;
    }
    micro_slope(g1, q.u, q.v, lam, real(0.5) / lam, k, a);
    micro_slope(g2, q.u, q.v, lam, real(0.5) / lam, k, b);
    MomAdj<real> lM;
    lM.zero();
    real la[4] = {0, 0, 0, 0}, lb[4] = {0, 0, 0, 0};
    real lt[4];
    real t[4];
    // Wc += r <psi>, Wcn += r <(a.psi) psi>, Wct += r <(b.psi) psi>
    mom_psi(M, 0, 0, t);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      lq.r += lWc[c] * t[c];
      lt[c] = q.r * lWc[c];
    }
    mom_psi_adj(M, 0, 0, lt, lM);
    mom_s_psi(M, a, 0, 0, t);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      lq.r += lWcn[c] * t[c];
      lt[c] = q.r * lWcn[c];
    }
    mom_s_psi_adj(M, a, 0, 0, lt, la, lM);
    mom_s_psi(M, b, 0, 0, t);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      lq.r += lWct[c] * t[c];
      lt[c] = q.r * lWct[c];
    }
    mom_s_psi_adj(M, b, 0, 0, lt, lb, lM);
    // Flr += r <u psi>, Malr += r (<(a.psi) u^2 psi> + <(b.psi) u v psi>)
    mom_psi(M, 1, 0, t);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      lq.r += lFlr[c] * t[c];
      lt[c] = q.r * lFlr[c];
    }
    mom_psi_adj(M, 1, 0, lt, lM);
    real t2[4];
    mom_s_psi(M, a, 2, 0, t);
    mom_s_psi(M, b, 1, 1, t2);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      lq.r += lMalr[c] * (t[c] + t2[c]);
      lt[c] = q.r * lMalr[c];
    }
    mom_s_psi_adj(M, a, 2, 0, lt, la, lM);
    mom_s_psi_adj(M, b, 1, 1, lt, lb, lM);
    real lU = real(0), lV = real(0), llam = real(0);
    real lg1[4] = {0, 0, 0, 0}, lg2[4] = {0, 0, 0, 0};
    micro_slope_adj(g1, q.u, q.v, lam, k, la, lg1, lU, lV, llam);
    micro_slope_adj(g2, q.u, q.v, lam, k, lb, lg2, lU, lV, llam);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      lwn[c] += lg1[c] * q.ir;
      lwt[c] += lg2[c] * q.ir;
      lq.ir += lg1[c] * wn[c] + lg2[c] * wt[c];
    }
    maxwell_moments_adj(M, side == 0 ? 1 : -1, k, lM, lU, lV, llam);
    lq.u += lU;
    lq.v += lV;
    // lam = r / (2 p)
    lq.r += llam * real(0.5) / q.p;
    lq.p += -llam * lam / q.p;
  }
}

template <class real>
DFW_HD void gks_flux_adj(const real* wl, const real* wln, const real* wlt, const real* wr, const real* wrn,
                         const real* wrt, const Prim<real>& ql, const Prim<real>& qr, real dt, const Coef<real>& k,
                         const real* lF, const real* lFt, real* lwl, real* lwln, real* lwlt, real* lwr, real* lwrn,
                         real* lwrt, PrimAdj<real>& lql, PrimAdj<real>& lqr) {
  GksEqAdj<real> e;
  gks_flux_adj_eq(wln, wlt, wrn, wrt, ql, qr, dt, k, lF, lFt, e);
  gks_flux_adj_sides(wln, wlt, wrn, wrt, ql, qr, k, e, lwln, lwlt, lwrn, lwrt, lql, lqr);
  (void)wl;
  (void)wr;
  (void)lwl;
  (void)lwr;
}

// ------------------------------------------------------------------------------------------------
// One side of the normal sweep and of an interface segment, forward and reverse.
//
// The interface kernels split the work of an interface segment over two threads, one per side:
// side 0 reconstructs cell f-1 (left state), side 1 cell f (right state).  The two sides share the
// characteristic basis of the segment (cells f-1 and f); they meet only in the flux and DF of each
// Gauss point and in the adjoint of the basis.
// ------------------------------------------------------------------------------------------------

// Normal sweep, one side.  cs[0..4]: the side's stencil, ordered away from the interface's far
// side (side 0: cells f-3..f+1; side 1: cells f+2..f-2); (a_lo, a_c, a_hi) the DF of the stencil's
// cells 1..3 in the same order; sgn_inv_dn = +1/dn (side 0) or -1/dn (side 1).  Gives the line
// value w and its normal derivative wn.
template <int RULE = -1, class real>
DFW_HD void normal_side(const Basis<real>& B, const real (*cs)[4], real a_lo, real a_c, real a_hi, real sgn_inv_dn,
                        const Coef<real>& k, real* w, real* wn) {
  real Q[5][4];
#pragma unroll
  for (int m = 0; m < 5; ++m) project(B, cs[m], Q[m]);
  real q[4], qd[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    real s[5], P2[2];
#pragma unroll
    for (int m = 0; m < 5; ++m) s[m] = Q[m][c];
    recon_poly<real, 2, RULE>(s, a_lo, a_c, a_hi, k, P2);
    q[c] = P2[0];
    qd[c] = P2[1] * sgn_inv_dn;
  }
  unproject(B, q, w);
  unproject(B, qd, wn);
}

// Reverse of normal_side; cell(m, c) gives component c of stencil cell m.  The stencil cells'
// adjoints go to lc_add(m, c, v) (add v to cell m, component c); the basis adjoint lB and la_c (the
// DF of the reconstructed cell, DF branch only) accumulate.  One characteristic component at a time: its projection, reconstruction forward and
// backward, and its share of the projection adjoints, so that only one chain is live.
template <int C, int RULE, class real, class CellFn, class AddFn>
DFW_HD void normal_side_adj_comp(const Basis<real>& B, CellFn cell, real a_lo, real a_c, real a_hi, real sgn_inv_dn,
                                 const Coef<real>& k, const real* lw, const real* lwn, real lqc, real lqdc,
                                 AddFn lc_add, BasisAdj<real>& lB, real& la_c) {
  real s[5], P2[2], lP[2], lQc[5] = {0, 0, 0, 0, 0};
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    real w[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) w[c] = cell(m, c);
    s[m] = project_comp<C>(B, w);
  }
  lP[0] = lqc;
  lP[1] = lqdc * sgn_inv_dn;
  recon_poly_adj<real, 2, RULE>(s, a_lo, a_c, a_hi, k, lP, lQc, la_c, P2);
  unproject_adj_B_comp<C>(B, P2[0], lw, lB);
  unproject_adj_B_comp<C>(B, P2[1] * sgn_inv_dn, lwn, lB);
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    real w[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) w[c] = cell(m, c);
    real d[4] = {0, 0, 0, 0};
    project_adj_comp<C>(B, w, lQc[m], d, lB);
#pragma unroll
    for (int c = 0; c < 4; ++c) lc_add(m, c, d[c]);
  }
}

// cell(m, c) is read once per component; callers that keep the cells in memory pass a reader that
// reloads them, so that nothing but the accumulators lives from one component to the next.
template <int RULE = -1, class real, class CellFn, class AddFn>
DFW_HD void normal_side_adj(const Basis<real>& B, CellFn cell, real a_lo, real a_c, real a_hi, real sgn_inv_dn,
                            const Coef<real>& k, const real* lw, const real* lwn, AddFn lc_add, BasisAdj<real>& lB,
                            real& la_c) {
  normal_side_adj_comp<0, RULE>(B, cell, a_lo, a_c, a_hi, sgn_inv_dn, k, lw, lwn, unproject_adj_q_comp<0>(B, lw),
                          unproject_adj_q_comp<0>(B, lwn), lc_add, lB, la_c);
  normal_side_adj_comp<1, RULE>(B, cell, a_lo, a_c, a_hi, sgn_inv_dn, k, lw, lwn, unproject_adj_q_comp<1>(B, lw),
                          unproject_adj_q_comp<1>(B, lwn), lc_add, lB, la_c);
  normal_side_adj_comp<2, RULE>(B, cell, a_lo, a_c, a_hi, sgn_inv_dn, k, lw, lwn, unproject_adj_q_comp<2>(B, lw),
                          unproject_adj_q_comp<2>(B, lwn), lc_add, lB, la_c);
  normal_side_adj_comp<3, RULE>(B, cell, a_lo, a_c, a_hi, sgn_inv_dn, k, lw, lwn, unproject_adj_q_comp<3>(B, lw),
                          unproject_adj_q_comp<3>(B, lwn), lc_add, lB, la_c);
}

// Segment, one side: line(m, c) = component c of the side's line value on segment row m-2;
// al = DF of the side's cell on rows -1, 0, +1.  Gives the states and their tangential derivatives
// at the two Gauss points (as segment_fluxes computes them).
template <int RULE = -1, class real, class LineFn>
DFW_HD void segment_side(const Basis<real>& B, LineFn line, const real* al, real inv_dt, const Coef<real>& k,
                         real (*gw)[4], real (*gwt)[4]) {
  real Q[5][4];
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    real w[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) w[c] = line(m, c);
    project(B, w, Q[m]);
  }
  real qv[2][4], qd[2][4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    real s[5], v[2], d[2];
#pragma unroll
    for (int m = 0; m < 5; ++m) s[m] = Q[m][c];
    recon_gauss<real, RULE>(s, al[0], al[1], al[2], k, v, d);
    qv[0][c] = v[0];
    qv[1][c] = v[1];
    qd[0][c] = d[0] * inv_dt;
    qd[1][c] = d[1] * inv_dt;
  }
#pragma unroll
  for (int g = 0; g < 2; ++g) {
    unproject(B, qv[g], gw[g]);
    unproject(B, qd[g], gwt[g]);
  }
}

// Reverse of segment_side for the adjoints lgw, lgwt of the Gauss-point states, in two halves.
// First half, one characteristic component at a time: the reverse of the Gauss-point
// reconstruction gives the characteristic adjoints of the side's five line values, handed to
// put_q(C, m, v) (component C, row m); lB and la_c accumulate.
template <int C, int RULE, class real, class LineFn, class PutFn>
DFW_HD void segment_side_adj_q_comp(const Basis<real>& B, LineFn line, const real* al, real inv_dt,
                                    const Coef<real>& k, const real (*lgw)[4], const real (*lgwt)[4], real lqv0,
                                    real lqv1, real lqd0, real lqd1, PutFn put_q, BasisAdj<real>& lB, real& la_c) {
  real s[5], lQc[5] = {0, 0, 0, 0, 0};
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    real w[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) w[c] = line(m, c);
    s[m] = project_comp<C>(B, w);
  }
  const real lv[2] = {lqv0, lqv1}, ld[2] = {lqd0 * inv_dt, lqd1 * inv_dt};
  real v[2], d[2];
  recon_gauss_adj<real, RULE>(s, al[0], al[1], al[2], k, lv, ld, lQc, la_c, v, d);
  unproject_adj_B_comp<C>(B, v[0], lgw[0], lB);
  unproject_adj_B_comp<C>(B, v[1], lgw[1], lB);
  unproject_adj_B_comp<C>(B, d[0] * inv_dt, lgwt[0], lB);
  unproject_adj_B_comp<C>(B, d[1] * inv_dt, lgwt[1], lB);
#pragma unroll
  for (int m = 0; m < 5; ++m) put_q(C, m, lQc[m]);
}

template <int RULE = -1, class real, class LineFn, class PutFn>
DFW_HD void segment_side_adj_q(const Basis<real>& B, LineFn line, const real* al, real inv_dt, const Coef<real>& k,
                               const real (*lgw)[4], const real (*lgwt)[4], PutFn put_q, BasisAdj<real>& lB,
                               real& la_c) {
#define DFW_SEG_COMP(C)                                                                                          \
  segment_side_adj_q_comp<C, RULE>(B, line, al, inv_dt, k, lgw, lgwt, unproject_adj_q_comp<C>(B, lgw[0]),      \
                                   unproject_adj_q_comp<C>(B, lgw[1]), unproject_adj_q_comp<C>(B, lgwt[0]),    \
                                   unproject_adj_q_comp<C>(B, lgwt[1]), put_q, lB, la_c)
  DFW_SEG_COMP(0);
  DFW_SEG_COMP(1);
  DFW_SEG_COMP(2);
  DFW_SEG_COMP(3);
#undef DFW_SEG_COMP
}

// Second half, one row at a time: the adjoint lw of line value w from the characteristic adjoints
// lq[0..3] of its four components (the projection's reverse); lB accumulates.
template <class real>
DFW_HD void segment_side_adj_line(const Basis<real>& B, const real* w, const real* lq, real* lw, BasisAdj<real>& lB) {
#pragma unroll
  for (int c = 0; c < 4; ++c) lw[c] = real(0);
  project_adj_comp<0>(B, w, lq[0], lw, lB);
  project_adj_comp<1>(B, w, lq[1], lw, lB);
  project_adj_comp<2>(B, w, lq[2], lw, lB);
  project_adj_comp<3>(B, w, lq[3], lw, lB);
}

// The whole reverse: the adjoints of the side's line values go to ll_add(m, c, v); lB and la_c
// accumulate.
template <int RULE = -1, class real, class LineFn, class AddFn>
DFW_HD void segment_side_adj(const Basis<real>& B, LineFn line, const real* al, real inv_dt, const Coef<real>& k,
                             const real (*lgw)[4], const real (*lgwt)[4], AddFn ll_add, BasisAdj<real>& lB,
                             real& la_c) {
  real lQ[5][4];
  segment_side_adj_q<RULE>(B, line, al, inv_dt, k, lgw, lgwt, [&](int C, int m, real v) { lQ[m][C] = v; }, lB, la_c);
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    real w[4], d[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) w[c] = line(m, c);
    segment_side_adj_line(B, w, lQ[m], d, lB);
#pragma unroll
    for (int c = 0; c < 4; ++c) ll_add(m, c, d[c]);
  }
}

// Reverse of the flux, its time derivative and the DF at one Gauss point (left state wl with normal
// and tangential derivatives wln, wlt; right state likewise): lF, lFt are the adjoints of the
// Gauss point's flux and time derivative, ldf that of its DF value.  Outputs accumulate.
template <class real, int FLUX>
DFW_HD void gp_flux_adj(const real* wl, const real* wln, const real* wlt, const real* wr, const real* wrn,
                        const real* wrt, real dt, const Coef<real>& k, const real* lF, const real* lFt, real ldf,
                        real* lwl, real* lwln, real* lwlt, real* lwr, real* lwrn, real* lwrt) {
  const Prim<real> ql = prim(wl, k), qr = prim(wr, k);
  PrimAdj<real> lql, lqr;
  lql.zero();
  lqr.zero();
  if (FLUX == 0)
    lf_flux_adj(wl, wln, wlt, wr, wrn, wrt, ql, qr, k, lF, lFt, lwl, lwln, lwlt, lwr, lwrn, lwrt, lql, lqr);
  else
    gks_flux_adj(wl, wln, wlt, wr, wrn, wrt, ql, qr, dt, k, lF, lFt, lwl, lwln, lwlt, lwr, lwrn, lwrt, lql, lqr);
  df_factor_adj(ql, qr, ldf, lql, lqr);
  prim_adj(wl, ql, k, lql, lwl);
  prim_adj(wr, qr, k, lqr, lwr);
}

}  // namespace dfw
