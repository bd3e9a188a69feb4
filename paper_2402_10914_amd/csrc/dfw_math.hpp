// Device arithmetic of the S2O4 DF-hybrid step (Zhang, Ji & Xu, arXiv:2402.10914), hand-expanded
// for gfx950.  Every function works in the local frame of an interface: component 1 is the normal
// momentum, component 2 the tangential one (y-interfaces swap rho*U and rho*V before calling,
// an exact reflection of the paper's rotation by pi/2, Section 2.1).
//
// Functions are __host__ __device__ so that the same arithmetic can be instantiated on the host
// with a counting scalar to obtain exact operation counts.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#define DFW_HD __host__ __device__ __forceinline__

namespace dfw {

// Reciprocal of a positive, finite, normal number (the WENO-Z denominators: products of the
// b_k + eps, at least eps^4, and sums of positive weights).  On the device: the hardware reciprocal estimate refined by Newton-Raphson steps in fused
// form, e = 1 - x r, r <- r + r e (two steps in FP64, one in FP32), within one unit in the last
// place of 1/x, in 5 (FP64) or 3 (FP32) instructions instead of the ten-instruction IEEE division
// sequence, whose scaling and fix-up steps only matter for zero, infinite or subnormal operands.
// On the host (operation counts, host-side checks): the plain division.
DFW_HD double rcp_pos(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
#else
  return 1.0 / x;
#endif
}

DFW_HD float rcp_pos(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  const float r = __builtin_amdgcn_rcpf(x);
  return fmaf(r, fmaf(-x, r, 1.0f), r);
#else
  return 1.0f / x;
#endif
}

template <class real>
DFW_HD real rcp_pos(real x) {
  return real(1) / x;
}

// Scheme constants in the working precision, converted once per kernel from the host values.
template <class real>
struct Coef {
  real gamma, gm1, inv_gm1, alpha_thres, eps, c1, c2, K;
  real d[4];      // WENO-AO linear weights d0..d3 (Section 3.1)
  real dr[3];     // d_k / d_3
  real inv_d3;
  real K2, k4K2;  // K + 2 and 4 / (K + 2)
  int sw_rule;    // hybrid switch: 0 max of the three DF values (eq. (42)), 1 their min, 2 the cell's own
};

// Eq. (42): the DF quadratic replaces WENO-AO for a cell when the largest DF value of the cell and
// its two neighbours along the sweep is below the threshold (strict).  Readings kept as options:
// sw_rule 1 takes the smallest of the three (a discontinuity in any of them), 2 the cell's own value.
// RULE >= 0 fixes the rule at compile time (for kernels at the register limit, where a rule read at
// run time costs spills); RULE < 0 reads k.sw_rule.
template <int RULE = -1, class real>
DFW_HD bool df_switch(real a_lo, real a_c, real a_hi, const Coef<real>& k) {
  const int rule = RULE >= 0 ? RULE : k.sw_rule;
  real mx = a_lo > a_c ? a_lo : a_c;
  mx = mx > a_hi ? mx : a_hi;
  real mn = a_lo < a_c ? a_lo : a_c;
  mn = mn < a_hi ? mn : a_hi;
  const real a = rule == 1 ? mn : (rule == 2 ? a_c : mx);
  return a < k.alpha_thres;
}

// ------------------------------------------------------------------------------------------------
// Characteristic basis (eigenvectors of the normal flux Jacobian at the arithmetic mean of the two
// cells beside the interface).  Right eigenvectors (columns): (1,u-c,v,H-uc), (1,u,v,q2/2),
// (0,0,1,v), (1,u+c,v,H+uc).  The left eigenvectors are applied in a factored closed form:
// with b1 = (gamma-1)/c^2, b2 = b1 q2/2 and T = b2 w0 - b1 (u w1 + v w2 - w3), s = (u w0 - w1)/c:
//   Q0 = (T + s)/2, Q1 = w0 - T, Q2 = w2 - v w0, Q3 = (T - s)/2.
// ------------------------------------------------------------------------------------------------
template <class real>
struct Basis {
  real u, v, c, ic, H, hq2, b1, b2;
};

template <class real>
DFW_HD Basis<real> make_basis(const real* wa, const real* wb, const Coef<real>& k) {
  Basis<real> B;
  const real h = real(0.5);
  real r = h * (wa[0] + wb[0]);
  real m = h * (wa[1] + wb[1]);
  real n = h * (wa[2] + wb[2]);
  real e = h * (wa[3] + wb[3]);
  real ir = real(1) / r;
  B.u = m * ir;
  B.v = n * ir;
  B.hq2 = h * (B.u * B.u + B.v * B.v);
  real p = k.gm1 * (e - r * B.hq2);
  real c2 = k.gamma * p * ir;
  B.c = sqrt(c2);
  B.ic = real(1) / B.c;
  B.H = (e + p) * ir;
  B.b1 = k.gm1 * (B.ic * B.ic);  // (gamma - 1) / c^2 from the reciprocal already formed
  B.b2 = B.hq2 * B.b1;
  return B;
}

template <class real>
DFW_HD void project(const Basis<real>& B, const real* w, real* q) {
  real T = B.b2 * w[0] - B.b1 * (B.u * w[1] + B.v * w[2] - w[3]);
  real s = (B.u * w[0] - w[1]) * B.ic;
  q[0] = real(0.5) * (T + s);
  q[1] = w[0] - T;
  q[2] = w[2] - B.v * w[0];
  q[3] = real(0.5) * (T - s);
}

template <class real>
DFW_HD void unproject(const Basis<real>& B, const real* q, real* w) {
  real w0 = q[0] + q[1] + q[3];
  real dq = q[3] - q[0];
  w[0] = w0;
  w[1] = B.u * w0 + B.c * dq;
  w[2] = B.v * w0 + q[2];
  w[3] = B.H * (q[0] + q[3]) + B.u * B.c * dq + B.hq2 * q[1] + B.v * q[2];
}

// The variables the reconstruction works on: characteristic (CHAR) or, as an ablation of that
// choice, the conservative variables themselves (component-wise reconstruction).
template <bool CHAR, class real>
DFW_HD void to_recon(const Basis<real>& B, const real* w, real* q) {
  if constexpr (CHAR) {
    project(B, w, q);
  } else {
#pragma unroll
    for (int c = 0; c < 4; ++c) q[c] = w[c];
  }
}

template <bool CHAR, class real>
DFW_HD void from_recon(const Basis<real>& B, const real* q, real* w) {
  if constexpr (CHAR) {
    unproject(B, q, w);
  } else {
#pragma unroll
    for (int c = 0; c < 4; ++c) w[c] = q[c];
  }
}

template <bool CHAR, class real>
DFW_HD Basis<real> recon_basis(const real* wa, const real* wb, const Coef<real>& k) {
  if constexpr (CHAR) {
    return make_basis(wa, wb, k);
  } else {
    return Basis<real>{};
  }
}

// ------------------------------------------------------------------------------------------------
// Hybrid reconstruction of one cell (Section 3.1 and 3.3).  Q[0..4] = Q_{i-2..i+2}; the result is
// the polynomial P(xi) = sum_n P[n] xi^n on the cell, xi = (x - x_{i+1/2})/dx in [-1, 0].
//   WENO-AO: P = sum_{k<3} (wb_k - wb_3 d_k/d_3) p_k + (wb_3/d_3) p_3 with WENO-Z weights.
//   DF branch (max of the three alphas < threshold): P = Q_i + alpha_i (p_1 - Q_i), which is the
//   paper's zero-mean quadratic with x0 = -dx/2, x1 = dx^2/3 written through p_1.
// NDEG limits the coefficients produced (2 = value and slope at the edge only).
// ------------------------------------------------------------------------------------------------
// Smoothness indicators beta_0..beta_3 of eq. (38) of the four WENO-AO stencils of a cell (five
// averages Q[0..4] = Q_{i-2..i+2}): Jiang-Shu forms for the three quadratics, closed form for the
// quartic.  The differences they are built from are kept, since they also determine the candidate
// polynomials: t_k is the second difference of stencil k (twice the xi^2 coefficient of p_k), s_k
// twice the slope of p_k at the cell centre (with the sign of its Jiang-Shu form: +p_0', -p_1',
// -p_2'), and u_1..u_4 the coefficients of the quartic in its Legendre-type basis on the cell: in
// zeta = xi + 1/2 its zeta^1..zeta^4 coefficients are u_1 - 3/20 u_3, u_2 - 3/14 u_4, u_3 and u_4.
// ------------------------------------------------------------------------------------------------
template <class real>
struct WenoTerms {
  real b[4];
  real t0, t1, t2, s0, s1, s2, u1, u2, u3, u4;
};

template <class real>
DFW_HD WenoTerms<real> weno_terms(const real* Q) {
  const real Q0 = Q[0], Q1 = Q[1], Q2 = Q[2], Q3 = Q[3], Q4 = Q[4];
  const real k1312 = real(13.0 / 12.0), k14 = real(0.25);
  WenoTerms<real> T;
  T.t0 = Q0 - real(2) * Q1 + Q2;
  T.t1 = Q1 - real(2) * Q2 + Q3;
  T.t2 = Q2 - real(2) * Q3 + Q4;
  T.s0 = Q0 - real(4) * Q1 + real(3) * Q2;
  T.s1 = Q1 - Q3;
  T.s2 = T.t2 - real(2) * (Q3 - Q2);  // 3 Q2 - 4 Q3 + Q4
  T.b[0] = k1312 * T.t0 * T.t0 + k14 * T.s0 * T.s0;
  T.b[1] = k1312 * T.t1 * T.t1 + k14 * T.s1 * T.s1;
  T.b[2] = k1312 * T.t2 * T.t2 + k14 * T.s2 * T.s2;
  // the quartic's coefficients from the same differences (exact identities of its cell-average fit)
  const real d40 = Q4 - Q0;
  T.u1 = (real(-11) * d40 - real(82) * T.s1) * real(1.0 / 120.0);
  T.u2 = (real(34) * T.t1 - real(3) * (T.t0 + T.t2)) * real(1.0 / 56.0);
  T.u3 = (real(2) * T.s1 + d40) * real(1.0 / 12.0);
  T.u4 = (T.t0 - real(2) * T.t1 + T.t2) * real(1.0 / 24.0);
  const real e1 = T.u1 + real(0.1) * T.u3;
  const real e2 = T.u2 + real(123.0 / 455.0) * T.u4;
  T.b[3] = e1 * e1 + real(13.0 / 3.0) * e2 * e2 + real(781.0 / 20.0) * T.u3 * T.u3 +
           real(1421461.0 / 2275.0) * T.u4 * T.u4;
  return T;
}

template <class real>
DFW_HD void weno_indicators(const real* Q, real* b) {
  const WenoTerms<real> T = weno_terms(Q);
#pragma unroll
  for (int q = 0; q < 4; ++q) b[q] = T.b[q];
}

// ------------------------------------------------------------------------------------------------
// Non-linear time limiter (Section 2.2, eqs. (27)-(29)).  Weight of one reconstruction:
//   a1 = 1 + (tau_Z / (beta_min + eps))^2,  a2 = 1 + (tau_Z / (beta_max + eps))^2,
//   alpha = 2 a2 / (a1 + a2)  (in (0, 1]: 1 on smooth data, -> 0 across a jump),
// beta_min, beta_max over the four indicators of eq. (38), tau_Z of eq. (37).  The weight of an
// interface is the smallest over the characteristic components of the two normal reconstructions
// beside it; recon_poly hands it out of the normal sweep (from the ratios tau/(beta_k + eps) that
// its WENO-Z weights already hold, or from this function where the DF branch skips them).
// ------------------------------------------------------------------------------------------------
template <class real>
DFW_HD real time_limiter_weight(const real* Q, const Coef<real>& k) {
  real b[4];
  weno_indicators(Q, b);
  const real tau = (fabs(b[3] - b[0]) + fabs(b[3] - b[1]) + fabs(b[3] - b[2])) * real(1.0 / 3.0);
  real bmin = b[0] < b[1] ? b[0] : b[1], bmax = b[0] > b[1] ? b[0] : b[1];
  bmin = bmin < b[2] ? bmin : b[2];
  bmin = bmin < b[3] ? bmin : b[3];
  bmax = bmax > b[2] ? bmax : b[2];
  bmax = bmax > b[3] ? bmax : b[3];
  const real x1 = tau / (bmin + k.eps), x2 = tau / (bmax + k.eps);
  const real a1 = real(1) + x1 * x1, a2 = real(1) + x2 * x2;
  return real(2) * a2 / (a1 + a2);
}

// ------------------------------------------------------------------------------------------------
// With om non-null it also stores the time-limiter weight of this stencil (eq. (29)).
template <class real, int NDEG, int RULE = -1>
DFW_HD void recon_poly(const real* Q, real a_lo, real a_c, real a_hi, const Coef<real>& k, real* P,
                       real* om = nullptr) {
  const real Q1 = Q[1], Q2 = Q[2], Q3 = Q[3];
  // candidate p1 (centred quadratic): coefficients of 1, xi, xi^2
  real p1_0 = (real(5) * Q2 + real(2) * Q3 - Q1) * real(1.0 / 6.0);
  real p1_1 = Q3 - Q2;
  real p1_2 = real(0.5) * (Q1 + Q3) - Q2;
  if (df_switch<RULE>(a_lo, a_c, a_hi, k)) {
    P[0] = Q2 + a_c * (p1_0 - Q2);
    if (NDEG > 1) P[1] = a_c * p1_1;
    if (NDEG > 2) P[2] = a_c * p1_2;
    if (NDEG > 3) P[3] = real(0);
    if (NDEG > 4) P[4] = real(0);
    if (om) *om = time_limiter_weight(Q, k);
    return;
  }
  const WenoTerms<real> T = weno_terms(Q);
  const real b0 = T.b[0], b1 = T.b[1], b2 = T.b[2], b3 = T.b[3];
  // WENO-Z weights, eqs. (36)-(37)
  real tau = (fabs(b3 - b0) + fabs(b3 - b1) + fabs(b3 - b2)) * real(1.0 / 3.0);
  // r_q = tau / (b_q + eps) from products of the B_q and few reciprocals: one of B0 B1 B2 B3 in
  // FP64 (a product of four numbers in [eps, 1e75] stays normal), 1/(B0 B1) and 1/(B2 B3) in FP32
  const real B0 = b0 + k.eps, B1 = b1 + k.eps, B2 = b2 + k.eps, B3 = b3 + k.eps;
  const real P01 = B0 * B1, P23 = B2 * B3;
  real r0, r1, r2, r3;
  if constexpr (std::is_same<real, float>::value) {
    const real i01 = rcp_pos(P01), i23 = rcp_pos(P23);
    r0 = tau * (B1 * i01), r1 = tau * (B0 * i01), r2 = tau * (B3 * i23), r3 = tau * (B2 * i23);
  } else {
    const real ti = tau * rcp_pos(P01 * P23);
    const real t23 = ti * P23, t01 = ti * P01;
    r0 = t23 * B1, r1 = t23 * B0, r2 = t01 * B3, r3 = t01 * B2;
  }
  if (om) {  // tau/(beta_min + eps) and tau/(beta_max + eps) are the largest and smallest ratio
    real rmax = r0 > r1 ? r0 : r1, rmin = r0 < r1 ? r0 : r1;
    rmax = rmax > r2 ? rmax : r2;
    rmax = rmax > r3 ? rmax : r3;
    rmin = rmin < r2 ? rmin : r2;
    rmin = rmin < r3 ? rmin : r3;
    const real a1 = real(1) + rmax * rmax, a2 = real(1) + rmin * rmin;
    *om = real(2) * a2 / (a1 + a2);
  }
  real w0 = k.d[0] * (real(1) + r0 * r0);
  real w1 = k.d[1] * (real(1) + r1 * r1);
  real w2 = k.d[2] * (real(1) + r2 * r2);
  real w3 = k.d[3] * (real(1) + r3 * r3);
  real iws = rcp_pos(w0 + w1 + w2 + w3);
  real g3 = w3 * iws;
  real g0 = w0 * iws - g3 * k.dr[0];
  real g1 = w1 * iws - g3 * k.dr[1];
  real g2 = w2 * iws - g3 * k.dr[2];
  real h3 = g3 * k.inv_d3;
  // Coefficients of xi^1..xi^4 of the candidates, written through the indicator terms (exact
  // identities of the cell-average fits): p_k has xi^2 coefficient t_k/2; p_0 has slope
  // (s_0 + t_0)/2 at the edge, p_1 and p_2 both Q3 - Q2; the quartic p_3 has c_4 = u_4,
  // c_3 = u_3 + 2 u_4, c_2 = u_2 + 3/2 u_3 + 9/7 u_4, c_1 = u_1 + u_2 + 3/5 u_3 + 2/7 u_4.
  const real p0_1 = real(0.5) * (T.s0 + T.t0);
  const real c1 = T.u1 + T.u2 + real(0.6) * T.u3 + real(2.0 / 7.0) * T.u4;
  const real c2 = T.u2 + real(1.5) * T.u3 + real(9.0 / 7.0) * T.u4;
  const real c3 = T.u3 + real(2) * T.u4;
  const real P1 = g0 * p0_1 + (g1 + g2) * p1_1 + h3 * c1;
  const real P2 = real(0.5) * (g0 * T.t0 + g1 * T.t1 + g2 * T.t2) + h3 * c2;
  const real P3 = h3 * c3, P4 = h3 * T.u4;
  // Every candidate has the cell average Q_i and g0 + g1 + g2 + h3 = 1, so the combination does
  // too; its value at the edge follows from that condition: the mean of xi^n over [-1, 0] is
  // (-1)^n / (n + 1).
  P[0] = Q2 + real(0.5) * P1 - real(1.0 / 3.0) * P2 + real(0.25) * P3 - real(0.2) * P4;
  if (NDEG > 1) P[1] = P1;
  if (NDEG > 2) P[2] = P2;
  if (NDEG > 3) P[3] = P3;
  if (NDEG > 4) P[4] = P4;
}

// Gauss points of a segment [-1, 0] (in units of its length): -1/2 -+ kGpDelta, kGpDelta = sqrt(3)/6.
constexpr double kGpDelta = 0.28867513459481288225;

// The hybrid reconstruction of one cell evaluated at the two Gauss points of the segment, xi =
// -1/2 - kGpDelta and -1/2 + kGpDelta (the tangential sweep): values v[g] and slopes d[g] (per
// unit xi).  The same polynomial as recon_poly, taken in the centred variable zeta = xi + 1/2,
// where the Gauss points are zeta = -/+ delta, delta = kGpDelta, delta^2 = 1/12:
//   P = D0 + D1 zeta + ... + D4 zeta^4 with
//   D1 = (g0 s0 - g1 s1 - g2 s2)/2 + h3 (u1 - 3/20 u3),  D2 = (g0 t0 + g1 t1 + g2 t2)/2 + h3 (u2 - 3/14 u4),
//   D3 = h3 u3,  D4 = h3 u4,
// and D0 fixed by the cell mean (D0 = Q_i - D2/12 - D4/80), so that
//   v = Q_i - D4/180 -/+ delta (D1 + D3/12),   d = D1 + D3/4 -/+ delta (2 D2 + D4/3).
// DF branch: D1 = alpha_i (Q3 - Q1)/2, D2 = alpha_i t1/2, D3 = D4 = 0.
template <class real, int RULE = -1>
DFW_HD void recon_gauss(const real* Q, real a_lo, real a_c, real a_hi, const Coef<real>& k, real* v, real* d) {
  const real Q2 = Q[2];
  real D1, D2, D3 = real(0), D4 = real(0);
  if (df_switch<RULE>(a_lo, a_c, a_hi, k)) {
    D1 = a_c * (real(0.5) * (Q[3] - Q[1]));
    D2 = a_c * (real(0.5) * (Q[1] - real(2) * Q2 + Q[3]));
  } else {
    const WenoTerms<real> T = weno_terms(Q);
    const real b0 = T.b[0], b1 = T.b[1], b2 = T.b[2], b3 = T.b[3];
    const real tau = (fabs(b3 - b0) + fabs(b3 - b1) + fabs(b3 - b2)) * real(1.0 / 3.0);
    const real B0 = b0 + k.eps, B1 = b1 + k.eps, B2 = b2 + k.eps, B3 = b3 + k.eps;
    const real P01 = B0 * B1, P23 = B2 * B3;
    real r0, r1, r2, r3;
    if constexpr (std::is_same<real, float>::value) {
      const real i01 = rcp_pos(P01), i23 = rcp_pos(P23);
      r0 = tau * (B1 * i01), r1 = tau * (B0 * i01), r2 = tau * (B3 * i23), r3 = tau * (B2 * i23);
    } else {
      const real ti = tau * rcp_pos(P01 * P23);
      const real t23 = ti * P23, t01 = ti * P01;
      r0 = t23 * B1, r1 = t23 * B0, r2 = t01 * B3, r3 = t01 * B2;
    }
    const real w0 = k.d[0] * (real(1) + r0 * r0);
    const real w1 = k.d[1] * (real(1) + r1 * r1);
    const real w2 = k.d[2] * (real(1) + r2 * r2);
    const real w3 = k.d[3] * (real(1) + r3 * r3);
    const real iws = rcp_pos(w0 + w1 + w2 + w3);
    const real g3 = w3 * iws;
    const real g0 = w0 * iws - g3 * k.dr[0];
    const real g1 = w1 * iws - g3 * k.dr[1];
    const real g2 = w2 * iws - g3 * k.dr[2];
    const real h3 = g3 * k.inv_d3;
    D1 = real(0.5) * (g0 * T.s0 - g1 * T.s1 - g2 * T.s2) + h3 * (T.u1 - real(0.15) * T.u3);
    D2 = real(0.5) * (g0 * T.t0 + g1 * T.t1 + g2 * T.t2) + h3 * (T.u2 - real(3.0 / 14.0) * T.u4);
    D3 = h3 * T.u3;
    D4 = h3 * T.u4;
  }
  const real dl = real(kGpDelta);
  const real ev = Q2 - real(1.0 / 180.0) * D4, od = dl * (D1 + real(1.0 / 12.0) * D3);
  const real evd = D1 + real(0.25) * D3, odd = dl * (real(2) * D2 + real(1.0 / 3.0) * D4);
  v[0] = ev - od;
  v[1] = ev + od;
  d[0] = evd - odd;
  d[1] = evd + odd;
}


// ------------------------------------------------------------------------------------------------
// Primitive variables and the DF of one Gauss point (Section 3.2):
//   alpha = 1/(1 + D^2), D = |pl-pr|/pl + |pl-pr|/pr + (Ma_n^l - Ma_n^r)^2 + (Ma_t^l - Ma_t^r)^2.
// ------------------------------------------------------------------------------------------------
template <class real>
struct Prim {
  real r, ir, u, v, p, c;
};

template <class real>
DFW_HD Prim<real> prim(const real* w, const Coef<real>& k) {
  Prim<real> q;
  q.r = w[0];
  q.ir = real(1) / w[0];
  q.u = w[1] * q.ir;
  q.v = w[2] * q.ir;
  q.p = k.gm1 * (w[3] - real(0.5) * (w[1] * q.u + w[2] * q.v));
  q.c = sqrt(k.gamma * q.p * q.ir);
  return q;
}

template <class real>
DFW_HD real df_factor(const Prim<real>& L, const Prim<real>& R) {
  real jump = fabs(L.p - R.p);
  real icl = real(1) / L.c, icr = real(1) / R.c;
  real dn = L.u * icl - R.u * icr;
  real dt = L.v * icl - R.v * icr;
  real D = jump * (real(1) / L.p + real(1) / R.p) + dn * dn + dt * dt;
  return real(1) / (real(1) + D * D);
}

// ------------------------------------------------------------------------------------------------
// Lax-Friedrichs flux (Section 2.3) and its time derivative for S2O4: the left and right time
// derivatives come from the Euler equations in primitive form (Cauchy-Kovalevskaya),
//   rho_t = -(u rho_x + rho u_x + v rho_y + rho v_y),  u_t = -(u u_x + v u_y + p_x/rho),
//   v_t = -(u v_x + v v_y + p_y/rho),  p_t = -(u p_x + v p_y + gamma p (u_x + v_y)),
// and dF/dt = (F_t^l + F_t^r)/2 - s (W_t^r - W_t^l)/2 with the LF speed s held fixed.
// ------------------------------------------------------------------------------------------------
template <class real>
DFW_HD void euler_time_derivs(const real* w, const Prim<real>& q, const real* wx, const real* wy,
                              const Coef<real>& k, real* wt, real* ft) {
  real ke = real(0.5) * (q.u * q.u + q.v * q.v);
  real ux = (wx[1] - q.u * wx[0]) * q.ir, vx = (wx[2] - q.v * wx[0]) * q.ir;
  real px = k.gm1 * (wx[3] - q.u * wx[1] - q.v * wx[2] + ke * wx[0]);
  real uy = (wy[1] - q.u * wy[0]) * q.ir, vy = (wy[2] - q.v * wy[0]) * q.ir;
  real py = k.gm1 * (wy[3] - q.u * wy[1] - q.v * wy[2] + ke * wy[0]);
  real rt = -(q.u * wx[0] + q.r * ux + q.v * wy[0] + q.r * vy);
  real ut = -(q.u * ux + q.v * uy + px * q.ir);
  real vt = -(q.u * vx + q.v * vy + py * q.ir);
  real pt = -(q.u * px + q.v * py + k.gamma * q.p * (ux + vy));
  wt[0] = rt;
  wt[1] = rt * q.u + q.r * ut;
  wt[2] = rt * q.v + q.r * vt;
  wt[3] = pt * k.inv_gm1 + rt * ke + q.r * (q.u * ut + q.v * vt);
  ft[0] = wt[1];
  ft[1] = wt[1] * q.u + w[1] * ut + pt;
  ft[2] = wt[1] * q.v + w[1] * vt;
  ft[3] = ut * (w[3] + q.p) + q.u * (wt[3] + pt);
}

template <class real, bool WANT_F>
DFW_HD void lf_flux(const real* wl, const real* wlx, const real* wly, const real* wr, const real* wrx,
                    const real* wry, const Prim<real>& ql, const Prim<real>& qr, const Coef<real>& k,
                    real* F, real* Ft) {
  real sl = fabs(ql.u) + ql.c, sr = fabs(qr.u) + qr.c;
  real s = sl >= sr ? sl : sr;
  real hs = real(0.5) * s;
  if (WANT_F) {
    real Fl[4] = {wl[1], wl[1] * ql.u + ql.p, wl[2] * ql.u, ql.u * (wl[3] + ql.p)};
    real Fr[4] = {wr[1], wr[1] * qr.u + qr.p, wr[2] * qr.u, qr.u * (wr[3] + qr.p)};
#pragma unroll
    for (int c = 0; c < 4; ++c) F[c] = real(0.5) * (Fl[c] + Fr[c]) - hs * (wr[c] - wl[c]);
  }
  real wtl[4], ftl[4], wtr[4], ftr[4];
  euler_time_derivs(wl, ql, wlx, wly, k, wtl, ftl);
  euler_time_derivs(wr, qr, wrx, wry, k, wtr, ftr);
#pragma unroll
  for (int c = 0; c < 4; ++c) Ft[c] = real(0.5) * (ftl[c] + ftr[c]) - hs * (wtr[c] - wtl[c]);
}

// ------------------------------------------------------------------------------------------------
// Gas-kinetic flux (Sections 2.2 and 3.4), Euler case: physical tau = 0 outside the exponential,
// numerical tau_n = c1 dt + c2 |(pl-pr)/(pl+pr)| dt inside it.
// Moments <u^a v^b xi^2c> of a Maxwellian (normalised by rho) factorise as mu[a] mv[b] mx[c].
// ------------------------------------------------------------------------------------------------
template <class real>
struct Mom {
  real mu[7];  // u-moments 0..6 (full space, or one half space)
  real mv[6];  // v-moments 0..5 (full space)
  real mx[3];  // <xi^0>, <xi^2>, <xi^4>
  real U, V, lam, h;  // h = 1 / (2 lam)
};

template <class real>
DFW_HD void full_recursion(real* m, int from, int to, real U, real h) {
  // m[n+2] = U m[n+1] + (n+1) h m[n], h = 1/(2 lambda)
  for (int n = from; n + 2 <= to; ++n) m[n + 2] = U * m[n + 1] + real(n + 1) * h * m[n];
}

// side: 0 full space, +1 u > 0, -1 u < 0.  h = 1/(2 lam), which the callers form as p/rho from the
// reciprocal of the density they already hold (the same value as 0.5/lam, also for p = 0 and on
// failing states, without a division).
template <class real>
DFW_HD void maxwell_moments(real U, real V, real lam, real h, int side, const Coef<real>& k, Mom<real>& M) {
  M.U = U;
  M.V = V;
  M.lam = lam;
  M.h = h;
  if (side == 0) {
    M.mu[0] = real(1);
    M.mu[1] = U;
  } else {
    const real inv_sqrt_pi = real(0.56418958354775628695);
    real sl = sqrt(lam);
    real g = real(0.5) * exp(-lam * U * U) * inv_sqrt_pi / sl;
    if (side > 0) {
      M.mu[0] = real(0.5) * erfc(-sl * U);
      M.mu[1] = U * M.mu[0] + g;
    } else {
      M.mu[0] = real(0.5) * erfc(sl * U);
      M.mu[1] = U * M.mu[0] - g;
    }
  }
  full_recursion(M.mu, 0, 6, U, h);
  M.mv[0] = real(1);
  M.mv[1] = V;
  full_recursion(M.mv, 0, 5, V, h);
  M.mx[0] = real(1);
  M.mx[1] = k.K * h;
  M.mx[2] = k.K * (k.K + real(2)) * h * h;
}

template <class real>
DFW_HD void maxwell_moments(real U, real V, real lam, int side, const Coef<real>& k, Mom<real>& M) {
  maxwell_moments(U, V, lam, real(0.5) / lam, side, k, M);
}

template <class real>
DFW_HD real mom(const Mom<real>& M, int a, int b, int c) {
  return M.mu[a] * M.mv[b] * M.mx[c];
}

// <(s . psi) u^a v^b xi^2c>, s . psi = s0 + s1 u + s2 v + s3 (u^2 + v^2 + xi^2)/2.  With the v- and
// xi-moments folded first it is a three-term form in the u-moments,
//   <(s . psi) u^a v^b xi^2c> = A mu[a] + B mu[a+1] + C mu[a+2],
//   A = s0 mv[b] mx[c] + s2 mv[b+1] mx[c] + s3/2 (mv[b+2] mx[c] + mv[b] mx[c+1]),
//   B = s1 mv[b] mx[c],  C = s3/2 mv[b] mx[c],
// whose coefficients depend on (s, b, c) only: calls with the same slope and v-power share them.
template <class real>
struct SForm {
  real A, B, C;
};

template <class real>
DFW_HD SForm<real> s_form(const Mom<real>& M, const real* s, int b, int c) {
  const real vx = M.mv[b] * M.mx[c];
  const real hs3 = real(0.5) * s[3];
  SForm<real> f;
  f.A = s[0] * vx + s[2] * (M.mv[b + 1] * M.mx[c]) + hs3 * (M.mv[b + 2] * M.mx[c] + M.mv[b] * M.mx[c + 1]);
  f.B = s[1] * vx;
  f.C = hs3 * vx;
  return f;
}

template <class real>
DFW_HD real s_apply(const SForm<real>& f, const real* mu, int a) {
  return f.A * mu[a] + f.B * mu[a + 1] + f.C * mu[a + 2];
}

// <(s . psi) u^a v^b psi>  (4 components)
template <class real>
DFW_HD void mom_s_psi(const Mom<real>& M, const real* s, int a, int b, real* out) {
  const SForm<real> f0 = s_form(M, s, b, 0), f1 = s_form(M, s, b + 1, 0), f2 = s_form(M, s, b + 2, 0);
  const SForm<real> fx = s_form(M, s, b, 1);
  out[0] = s_apply(f0, M.mu, a);
  out[1] = s_apply(f0, M.mu, a + 1);
  out[2] = s_apply(f1, M.mu, a);
  out[3] = real(0.5) * (s_apply(f0, M.mu, a + 2) + s_apply(f2, M.mu, a) + s_apply(fx, M.mu, a));
}

// <u^a v^b psi>
template <class real>
DFW_HD void mom_psi(const Mom<real>& M, int a, int b, real* out) {
  out[0] = mom(M, a, b, 0);
  out[1] = mom(M, a + 1, b, 0);
  out[2] = mom(M, a, b + 1, 0);
  out[3] = real(0.5) * (mom(M, a + 2, b, 0) + mom(M, a, b + 2, 0) + mom(M, a, b, 1));
}

// Micro-slope s with <(s . psi) psi> = g (g = dW / rho), closed-form inverse of the moment matrix;
// h = 1 / (2 lam).
template <class real>
DFW_HD void micro_slope(const real* g, real U, real V, real lam, real h, const Coef<real>& k, real* s) {
  real B = U * U + V * V + k.K2 * h;
  real R4 = real(2) * g[3] - B * g[0];
  real R3 = g[2] - V * g[0];
  real R2 = g[1] - U * g[0];
  s[3] = k.k4K2 * (lam * lam) * (R4 - real(2) * U * R2 - real(2) * V * R3);
  s[2] = real(2) * lam * R3 - V * s[3];
  s[1] = real(2) * lam * R2 - U * s[3];
  s[0] = g[0] - U * s[1] - V * s[2] - real(0.5) * s[3] * B;
}

// GKS flux at one Gauss point.  wl/wr: states; wln/wrn: normal derivatives; wlt/wrt: tangential
// derivatives.  Outputs F (if WANT_F) and dF/dt by the S2O4 fit of eqs. (23)-(25) to the time
// integrals over dt and dt/2, written in closed form:
//   F    = cf1 Fc + cf2 (Ma_c - Ma_lr) + (1 - cf1) F_lr
//   F_t  = ct1 (Fc - F_lr) + ct2 (Ma_c - Ma_lr) + MA_c
// with E1 = exp(-dt/tau), E2 = exp(-dt/(2 tau)):
//   cf1 = 1 - (tau/dt)(3 - 4E2 + E1),  cf2 = (tau^2/dt)(3 - 4E2 + E1) + tau (E1 - 2E2),
//   ct1 = 4 tau (1 - E2)^2 / dt^2,     ct2 = 4 (tau dt E2 (1 - E2) - tau^2 (1 - E2)^2) / dt^2.
template <class real, bool WANT_F>
DFW_HD void gks_flux(const real* wl, const real* wln, const real* wlt, const real* wr, const real* wrn,
                     const real* wrt, const Prim<real>& ql, const Prim<real>& qr, real dt,
                     const Coef<real>& k, real* F, real* Ft) {
  real Wc[4] = {0, 0, 0, 0}, Wcn[4] = {0, 0, 0, 0}, Wct[4] = {0, 0, 0, 0};
  real Flr[4] = {0, 0, 0, 0}, Malr[4] = {0, 0, 0, 0};
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const real* w = side == 0 ? wl : wr;
    const real* wn = side == 0 ? wln : wrn;
    const real* wt = side == 0 ? wlt : wrt;
    const Prim<real>& q = side == 0 ? ql : qr;
    real lam = real(0.5) * q.r / q.p;
    Mom<real> M;
    maxwell_moments(q.u, q.v, lam, q.p * q.ir, side == 0 ? 1 : -1, k, M);
    real g[4], a[4], b[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) g[c] = wn[c] * q.ir;
    micro_slope(g, q.u, q.v, lam, M.h, k, a);
#pragma unroll
    for (int c = 0; c < 4; ++c) g[c] = wt[c] * q.ir;
    micro_slope(g, q.u, q.v, lam, M.h, k, b);
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
  // equilibrium state at the interface
  real irc = real(1) / Wc[0];
  real Uc = Wc[1] * irc, Vc = Wc[2] * irc;
  real pc = k.gm1 * (Wc[3] - real(0.5) * (Wc[1] * Uc + Wc[2] * Vc));
  real lamc = real(0.5) * Wc[0] / pc;
  Mom<real> M;
  maxwell_moments(Uc, Vc, lamc, pc * irc, 0, k, M);
  real g[4], ac[4], bc[4], Ac[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) g[c] = Wcn[c] * irc;
  micro_slope(g, Uc, Vc, lamc, M.h, k, ac);
#pragma unroll
  for (int c = 0; c < 4; ++c) g[c] = Wct[c] * irc;
  micro_slope(g, Uc, Vc, lamc, M.h, k, bc);
  // compatibility: <(A . psi) psi> = -<((a . psi) u + (b . psi) v) psi>
  real t1[4], t2[4];
  mom_s_psi(M, ac, 1, 0, t1);
  mom_s_psi(M, bc, 0, 1, t2);
#pragma unroll
  for (int c = 0; c < 4; ++c) g[c] = -(t1[c] + t2[c]);
  micro_slope(g, Uc, Vc, lamc, M.h, k, Ac);
  real Fc[4], Mac[4], MAc[4];
  mom_psi(M, 1, 0, Fc);
  mom_s_psi(M, ac, 2, 0, t1);
  mom_s_psi(M, bc, 1, 1, t2);
  mom_s_psi(M, Ac, 1, 0, MAc);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    Fc[c] *= Wc[0];
    Mac[c] = Wc[0] * (t1[c] + t2[c]);
    MAc[c] *= Wc[0];
  }
  // time coefficients
  real tau = k.c1 * dt + k.c2 * fabs((ql.p - qr.p) / (ql.p + qr.p)) * dt;
  real E2 = exp(-real(0.5) * dt / tau);
  real E1 = E2 * E2;
  real om = real(1) - E2;
  real idt = real(1) / dt;
  real ct1 = real(4) * tau * om * om * idt * idt;
  real ct2 = real(4) * (tau * dt * E2 * om - tau * tau * om * om) * idt * idt;
#pragma unroll
  for (int c = 0; c < 4; ++c) Ft[c] = ct1 * (Fc[c] - Flr[c]) + ct2 * (Mac[c] - Malr[c]) + MAc[c];
  if (WANT_F) {
    real z = real(3) - real(4) * E2 + E1;
    real cf1 = real(1) - tau * idt * z;
    real cf2 = tau * tau * idt * z + tau * (E1 - real(2) * E2);
#pragma unroll
    for (int c = 0; c < 4; ++c) F[c] = cf1 * Fc[c] + cf2 * (Mac[c] - Malr[c]) + (real(1) - cf1) * Flr[c];
  }
}

// ------------------------------------------------------------------------------------------------
// One interface segment, normal sweep (Section 3.1, Algorithm 1): from the six cells along the
// normal (cells f-3..f+2 around interface f) and the DF of cells f-2..f+1, the line values of the
// left state (cell f-1 at its right edge) and the right state (cell f at its left edge, mirrored
// stencil) and their normal derivatives, in conservative variables.
// ------------------------------------------------------------------------------------------------
template <class real, bool CHAR = true>
DFW_HD void normal_sweep(const real (*cell)[4], real a0, real a1, real a2, real a3, real inv_dn,
                         const Coef<real>& k, real* wl, real* wr, real* wln, real* wrn, real* om = nullptr) {
  const Basis<real> B = recon_basis<CHAR>(cell[2], cell[3], k);
  real Q[6][4];
#pragma unroll
  for (int m = 0; m < 6; ++m) to_recon<CHAR>(B, cell[m], Q[m]);
  real ql[4], qld[4], qr[4], qrd[4];
  real omin = real(1), wk = real(1);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    real s[5], P2[2];
#pragma unroll
    for (int m = 0; m < 5; ++m) s[m] = Q[m][c];
    recon_poly<real, 2>(s, a0, a1, a2, k, P2, om ? &wk : nullptr);
    if (om) omin = omin < wk ? omin : wk;
    ql[c] = P2[0];
    qld[c] = P2[1] * inv_dn;
#pragma unroll
    for (int m = 0; m < 5; ++m) s[m] = Q[5 - m][c];
    recon_poly<real, 2>(s, a3, a2, a1, k, P2, om ? &wk : nullptr);
    if (om) omin = omin < wk ? omin : wk;
    qr[c] = P2[0];
    qrd[c] = -P2[1] * inv_dn;
  }
  from_recon<CHAR>(B, ql, wl);
  from_recon<CHAR>(B, qr, wr);
  from_recon<CHAR>(B, qld, wln);
  from_recon<CHAR>(B, qrd, wrn);
  if (om) *om = omin;  // time-limiter weight of the interface (eq. (29)): both sides, all components
}

// ------------------------------------------------------------------------------------------------
// One interface segment, tangential sweep and fluxes: the basis of the segment from its two cells
// (wa, wb); line(side, m, c) returns component c of the side's line value on segment row m-2..m+2;
// alpha[side][0..2] are the DF of the same-side cells on rows -1, 0, +1.  Produces the sums over
// the two Gauss points of the flux and its time derivative (quadrature weights applied by the
// caller) and the product of the two Gauss-point DF values.
// ------------------------------------------------------------------------------------------------
template <class real, int FLUX, bool WANT_F, bool WANT_DF, bool CHAR = true, class LineFn>
DFW_HD void segment_fluxes(const real* wa, const real* wb, LineFn line, const real (*alpha)[3],
                           const real* wln, const real* wrn, real dt, real inv_dt, const Coef<real>& k,
                           real* Fs, real* Fts, real& dfp) {
  const Basis<real> B = recon_basis<CHAR>(wa, wb, k);
  real gw[2][2][4], gwt[2][2][4];  // [side][gauss point][component]
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    real Q[5][4];
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      real w[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) w[c] = line(side, m, c);
      to_recon<CHAR>(B, w, Q[m]);
    }
    real qv[2][4], qd[2][4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      real s[5], v[2], d[2];
#pragma unroll
      for (int m = 0; m < 5; ++m) s[m] = Q[m][c];
      recon_gauss<real>(s, alpha[side][0], alpha[side][1], alpha[side][2], k, v, d);
      qv[0][c] = v[0];
      qv[1][c] = v[1];
      qd[0][c] = d[0] * inv_dt;
      qd[1][c] = d[1] * inv_dt;
    }
#pragma unroll
    for (int g = 0; g < 2; ++g) {
      from_recon<CHAR>(B, qv[g], gw[side][g]);
      from_recon<CHAR>(B, qd[g], gwt[side][g]);
    }
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    Fs[c] = real(0);
    Fts[c] = real(0);
  }
  dfp = real(1);
#pragma unroll
  for (int g = 0; g < 2; ++g) {
    Prim<real> ql = prim(gw[0][g], k), qr = prim(gw[1][g], k);
    real F[4], Ft[4];
    if (FLUX == 0)
      lf_flux<real, WANT_F>(gw[0][g], wln, gwt[0][g], gw[1][g], wrn, gwt[1][g], ql, qr, k, F, Ft);
    else
      gks_flux<real, WANT_F>(gw[0][g], wln, gwt[0][g], gw[1][g], wrn, gwt[1][g], ql, qr, dt, k, F, Ft);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      if (WANT_F) Fs[c] += F[c];
      Fts[c] += Ft[c];
    }
    if (WANT_DF) dfp *= df_factor(ql, qr);
  }
}

}  // namespace dfw
