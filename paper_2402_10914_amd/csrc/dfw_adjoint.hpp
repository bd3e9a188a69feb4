// Hand-written reverse-mode (adjoint) counterparts of the device arithmetic in dfw_math.hpp.
//
// Convention: for y = f(x), f_adj(x, ..., ly, lx) adds (dy/dx)^T ly into lx (accumulates; callers
// zero the adjoint arrays).  Each adjoint recomputes the forward intermediates it needs from the
// primal inputs.  Kinks follow a fixed subgradient convention: d|x| = sign(x) with sign(0) = 0;
// max(a, b) routes to a when a >= b; the hybrid switch of eq. (34) has zero derivative (the branch
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

template <class real>
DFW_HD void unproject_adj(const Basis<real>& B, const real* q, const real* lw, real* lq, BasisAdj<real>& lB) {
  real w0 = q[0] + q[1] + q[3];
  real dq = q[3] - q[0];
  real lw0 = lw[0] + B.u * lw[1] + B.v * lw[2];
  real ldq = B.c * lw[1] + B.u * B.c * lw[3];
  lB.u += lw[1] * w0 + lw[3] * B.c * dq;
  lB.c += lw[1] * dq + lw[3] * B.u * dq;
  lB.v += lw[2] * w0 + lw[3] * q[2];
  lB.H += lw[3] * (q[0] + q[3]);
  lB.hq2 += lw[3] * q[1];
  lq[0] += lw0 - ldq + lw[3] * B.H;
  lq[1] += lw0 + lw[3] * B.hq2;
  lq[2] += lw[2] + lw[3] * B.v;
  lq[3] += lw0 + ldq + lw[3] * B.H;
}

// ------------------------------------------------------------------------------------------------
// Hybrid reconstruction: lP (NDEG coefficients) -> lQ (5) and the DF of the centre cell (DF branch).
// ------------------------------------------------------------------------------------------------
template <class real, int NDEG>
DFW_HD void recon_poly_adj(const real* Q, real a_lo, real a_c, real a_hi, const Coef<real>& k, const real* lP, real* lQ,
                           real& la_c) {
  const real Q0 = Q[0], Q1 = Q[1], Q2 = Q[2], Q3 = Q[3], Q4 = Q[4];
  const real i6 = real(1.0 / 6.0);
  real p1_0 = (real(5) * Q2 + real(2) * Q3 - Q1) * i6;
  real p1_1 = Q3 - Q2;
  real p1_2 = real(0.5) * (Q1 + Q3) - Q2;
  real lP0 = lP[0], lP1 = NDEG > 1 ? lP[1] : real(0), lP2 = NDEG > 2 ? lP[2] : real(0);
  real lP3 = NDEG > 3 ? lP[3] : real(0), lP4 = NDEG > 4 ? lP[4] : real(0);
  real amax = a_lo > a_c ? a_lo : a_c;
  amax = amax > a_hi ? amax : a_hi;
  real l10, l11, l12;  // adjoints of p1's coefficients
  if (amax < k.alpha_thres) {
    la_c += lP0 * (p1_0 - Q2) + lP1 * p1_1 + lP2 * p1_2;
    lQ[2] += lP0 * (real(1) - a_c);
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
    real r[4], w[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      r[q] = tau / be[q];
      w[q] = k.d[q] * (real(1) + r[q] * r[q]);
    }
    real iws = real(1) / (w[0] + w[1] + w[2] + w[3]);
    real g3 = w[3] * iws;
    real g0 = w[0] * iws - g3 * k.dr[0];
    real g1 = w[1] * iws - g3 * k.dr[1];
    real g2 = w[2] * iws - g3 * k.dr[2];
    real h3 = g3 * k.inv_d3;
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
      real lr = lw[q] * k.d[q] * real(2) * r[q];
      ltau += lr / be[q];
      lb[q] = -lr * r[q] / be[q];
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

template <class real>
DFW_HD void eval_poly_at_adj(real xi, real lval, real lder, real* lP) {
  real x2 = xi * xi, x3 = x2 * xi, x4 = x3 * xi;
  lP[0] += lval;
  lP[1] += lval * xi + lder;
  lP[2] += lval * x2 + lder * real(2) * xi;
  lP[3] += lval * x3 + lder * real(3) * x2;
  lP[4] += lval * x4 + lder * real(4) * x3;
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
  const real K2 = k.K + real(2);
  real B = U * U + V * V + K2 * real(0.5) / lam;
  real R4 = real(2) * g[3] - B * g[0];
  real R3 = g[2] - V * g[0];
  real R2 = g[1] - U * g[0];
  real kap = real(4) * lam * lam / K2;
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
  llam += ls3 * Z * real(8) * lam / K2;
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
  llam += -K2 * real(0.5) / (lam * lam) * lB;
}

// Adjoint of gks_flux (lF may be null when the flux itself was not requested).
template <class real>
DFW_HD void gks_flux_adj(const real* wl, const real* wln, const real* wlt, const real* wr, const real* wrn,
                         const real* wrt, const Prim<real>& ql, const Prim<real>& qr, real dt, const Coef<real>& k,
                         const real* lF, const real* lFt, real* lwl, real* lwln, real* lwlt, real* lwr, real* lwrn,
                         real* lwrt, PrimAdj<real>& lql, PrimAdj<real>& lqr) {
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
    micro_slope(g, q.u, q.v, lam, k, a);
#pragma unroll
    for (int c = 0; c < 4; ++c) g[c] = wt[c] * q.ir;
    micro_slope(g, q.u, q.v, lam, k, b);
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
  micro_slope(gn, Uc, Vc, lamc, k, ac);
  micro_slope(gt, Uc, Vc, lamc, k, bc);
  real y1[4], y2[4];
  mom_s_psi(Mc, ac, 1, 0, y1);
  mom_s_psi(Mc, bc, 0, 1, y2);
#pragma unroll
  for (int c = 0; c < 4; ++c) gA[c] = -(y1[c] + y2[c]);
  micro_slope(gA, Uc, Vc, lamc, k, Ac);
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
  real lFc[4], lFlr[4], lMac[4], lMalr[4], lMAc[4];
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
    lql.p += lpq * (real(1) - pq) * isum;
    lqr.p += lpq * (real(-1) - pq) * isum;
  }
  // ---- reverse: equilibrium-state fluxes
  MomAdj<real> lMc;
  lMc.zero();
  real lWc[4] = {0, 0, 0, 0}, lWcn[4] = {0, 0, 0, 0}, lWct[4] = {0, 0, 0, 0};
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
    micro_slope(g1, q.u, q.v, lam, k, a);
    micro_slope(g2, q.u, q.v, lam, k, b);
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
  (void)lwl;
  (void)lwr;
}

// ------------------------------------------------------------------------------------------------
// Segment and normal-sweep adjoints (reverse of segment_fluxes and normal_sweep).
// ------------------------------------------------------------------------------------------------
// Inputs as segment_fluxes plus the adjoints of its outputs (sums over the two Gauss points of
// the flux and its time derivative, and the Gauss-point DF product).  Outputs (accumulated):
// adjoints of the basis cells wa, wb, of the line values line(side, m, c) as ll[side][m][c], of the
// normal derivatives, and of the DF of the same-side centre cells la_c[side] (DF branch only).
template <class real, int FLUX, class LineFn>
DFW_HD void segment_fluxes_adj(const real* wa, const real* wb, LineFn line, const real (*alpha)[3], const real* wln,
                               const real* wrn, real dt, real inv_dt, const Coef<real>& k, const real* lFs,
                               const real* lFts, real ldfp, real* lwa, real* lwb, real (*ll)[5][4], real* lwln,
                               real* lwrn, real* la_c) {
  Basis<real> B = make_basis(wa, wb, k);
  real gw[2][2][4], gwt[2][2][4], qv[2][2][4], qd[2][2][4];
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    real Q[5][4];
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      real w[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) w[c] = line(side, m, c);
      project(B, w, Q[m]);
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      real s[5], Pc[5];
#pragma unroll
      for (int m = 0; m < 5; ++m) s[m] = Q[m][c];
      recon_poly<real, 5>(s, alpha[side][0], alpha[side][1], alpha[side][2], k, Pc);
      real v0, d0, v1, d1;
      eval_poly_at(Pc, real(kXiGp0), v0, d0);
      eval_poly_at(Pc, real(kXiGp1), v1, d1);
      qv[side][0][c] = v0;
      qv[side][1][c] = v1;
      qd[side][0][c] = d0 * inv_dt;
      qd[side][1][c] = d1 * inv_dt;
    }
#pragma unroll
    for (int g = 0; g < 2; ++g) {
      unproject(B, qv[side][g], gw[side][g]);
      unproject(B, qd[side][g], gwt[side][g]);
    }
  }
  // per Gauss point: flux and DF adjoints -> states
  real lgw[2][2][4], lgwt[2][2][4];
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int g = 0; g < 2; ++g)
#pragma unroll
      for (int c = 0; c < 4; ++c) lgw[s][g][c] = lgwt[s][g][c] = real(0);
  Prim<real> qg[2][2];
#pragma unroll
  for (int g = 0; g < 2; ++g) {
    qg[0][g] = prim(gw[0][g], k);
    qg[1][g] = prim(gw[1][g], k);
  }
  real dfg[2] = {df_factor(qg[0][0], qg[1][0]), df_factor(qg[0][1], qg[1][1])};
#pragma unroll
  for (int g = 0; g < 2; ++g) {
    PrimAdj<real> lql, lqr;
    lql.zero();
    lqr.zero();
    if (FLUX == 0)
      lf_flux_adj(gw[0][g], wln, gwt[0][g], gw[1][g], wrn, gwt[1][g], qg[0][g], qg[1][g], k, lFs, lFts, lgw[0][g], lwln,
                  lgwt[0][g], lgw[1][g], lwrn, lgwt[1][g], lql, lqr);
    else
      gks_flux_adj(gw[0][g], wln, gwt[0][g], gw[1][g], wrn, gwt[1][g], qg[0][g], qg[1][g], dt, k, lFs, lFts, lgw[0][g],
                   lwln, lgwt[0][g], lgw[1][g], lwrn, lgwt[1][g], lql, lqr);
    df_factor_adj(qg[0][g], qg[1][g], ldfp * dfg[1 - g], lql, lqr);
    prim_adj(gw[0][g], qg[0][g], k, lql, lgw[0][g]);
    prim_adj(gw[1][g], qg[1][g], k, lqr, lgw[1][g]);
  }
  // states at the Gauss points -> reconstruction -> line values
  BasisAdj<real> lB;
  lB.zero();
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    real lqv[2][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}}, lqd[2][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
#pragma unroll
    for (int g = 0; g < 2; ++g) {
      unproject_adj(B, qv[side][g], lgw[side][g], lqv[g], lB);
      unproject_adj(B, qd[side][g], lgwt[side][g], lqd[g], lB);
    }
    real Q[5][4], lQ[5][4];
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      real w[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        w[c] = line(side, m, c);
        lQ[m][c] = real(0);
      }
      project(B, w, Q[m]);
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      real s[5], lP[5] = {0, 0, 0, 0, 0}, lQc[5] = {0, 0, 0, 0, 0};
#pragma unroll
      for (int m = 0; m < 5; ++m) s[m] = Q[m][c];
      eval_poly_at_adj(real(kXiGp0), lqv[0][c], lqd[0][c] * inv_dt, lP);
      eval_poly_at_adj(real(kXiGp1), lqv[1][c], lqd[1][c] * inv_dt, lP);
      recon_poly_adj<real, 5>(s, alpha[side][0], alpha[side][1], alpha[side][2], k, lP, lQc, la_c[side]);
#pragma unroll
      for (int m = 0; m < 5; ++m) lQ[m][c] = lQc[m];
    }
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      real w[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) w[c] = line(side, m, c);
      project_adj(B, w, lQ[m], ll[side][m], lB);
    }
  }
  make_basis_adj(wa, wb, k, lB, lwa, lwb);
}

// Reverse of normal_sweep: lcell[6][4] accumulates, la1/la2 receive the DF of cells f-1 / f
// (the centre cells of the left / right reconstructions, DF branch only).
template <class real>
DFW_HD void normal_sweep_adj(const real (*cell)[4], real a0, real a1, real a2, real a3, real inv_dn, const Coef<real>& k,
                             const real* lwl, const real* lwr, const real* lwln, const real* lwrn, real (*lcell)[4],
                             real& la1, real& la2) {
  Basis<real> B = make_basis(cell[2], cell[3], k);
  real Q[6][4];
#pragma unroll
  for (int m = 0; m < 6; ++m) project(B, cell[m], Q[m]);
  real ql[4], qld[4], qr[4], qrd[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    real s[5], P2[2];
#pragma unroll
    for (int m = 0; m < 5; ++m) s[m] = Q[m][c];
    recon_poly<real, 2>(s, a0, a1, a2, k, P2);
    ql[c] = P2[0];
    qld[c] = P2[1] * inv_dn;
#pragma unroll
    for (int m = 0; m < 5; ++m) s[m] = Q[5 - m][c];
    recon_poly<real, 2>(s, a3, a2, a1, k, P2);
    qr[c] = P2[0];
    qrd[c] = -P2[1] * inv_dn;
  }
  BasisAdj<real> lB;
  lB.zero();
  real lql[4] = {0, 0, 0, 0}, lqld[4] = {0, 0, 0, 0}, lqr[4] = {0, 0, 0, 0}, lqrd[4] = {0, 0, 0, 0};
  unproject_adj(B, ql, lwl, lql, lB);
  unproject_adj(B, qr, lwr, lqr, lB);
  unproject_adj(B, qld, lwln, lqld, lB);
  unproject_adj(B, qrd, lwrn, lqrd, lB);
  real lQ[6][4];
#pragma unroll
  for (int m = 0; m < 6; ++m)
#pragma unroll
    for (int c = 0; c < 4; ++c) lQ[m][c] = real(0);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    real s[5], lP[2], lQc[5];
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      s[m] = Q[m][c];
      lQc[m] = real(0);
    }
    lP[0] = lql[c];
    lP[1] = lqld[c] * inv_dn;
    recon_poly_adj<real, 2>(s, a0, a1, a2, k, lP, lQc, la1);
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      lQ[m][c] += lQc[m];
      s[m] = Q[5 - m][c];
      lQc[m] = real(0);
    }
    lP[0] = lqr[c];
    lP[1] = -lqrd[c] * inv_dn;
    recon_poly_adj<real, 2>(s, a3, a2, a1, k, lP, lQc, la2);
#pragma unroll
    for (int m = 0; m < 5; ++m) lQ[5 - m][c] += lQc[m];
  }
#pragma unroll
  for (int m = 0; m < 6; ++m) project_adj(B, cell[m], lQ[m], lcell[m], lB);
  make_basis_adj(cell[2], cell[3], k, lB, lcell[2], lcell[3]);
}

}  // namespace dfw
