// Host check of the reconstruction forms of dfw_math.hpp (the kernels' own __host__ __device__
// functions, run on the host in FP64).  Prints one line per property: name, worst deviation
// relative to max |Q|.  Built and run by tests/test_recon_forms.py.
//   gauss_vs_poly   recon_gauss against recon_poly<5> evaluated at xi = -1/2 -/+ sqrt(3)/6
//                   (values and slopes), both branches of the hybrid switch
//   cell_mean       the recon_poly<5> polynomial has the cell average Q_i over xi in [-1, 0]
//   edge_vs_poly    recon_poly<2> (value and slope at xi = 0) against recon_poly<5>
//   indicators      weno_terms' beta_0..beta_2 against the Jiang-Shu forms written from the
//                   candidate polynomials' derivatives at the cell centre
//   quadratic       cell averages of a quadratic are reconstructed exactly (value and slope at
//                   the edge and at the Gauss points)
#include <cmath>
#include <cstdio>
#include <random>

#include "../paper_2402_10914_amd/csrc/dfw_math.hpp"

using namespace dfw;

static Coef<double> coef(double thres) {
  Coef<double> k;
  const double g = 1.4, dh = 0.85, dl = 0.85;
  k.gamma = g; k.gm1 = g - 1; k.inv_gm1 = 1 / (g - 1); k.alpha_thres = thres; k.eps = 1e-6;
  k.c1 = 0.01; k.c2 = 5.0; k.K = (4 - 2 * g) / (g - 1);
  const double d[4] = {(1 - dh) * (1 - dl) / 2, (1 - dh) * dl, (1 - dh) * (1 - dl) / 2, dh};
  for (int i = 0; i < 4; ++i) k.d[i] = d[i];
  for (int i = 0; i < 3; ++i) k.dr[i] = d[i] / d[3];
  k.inv_d3 = 1 / d[3]; k.K2 = k.K + 2; k.k4K2 = 4 / (k.K + 2); k.sw_rule = 0;
  return k;
}

static void poly_at(const double* P, double x, double& v, double& d) {
  v = (((P[4] * x + P[3]) * x + P[2]) * x + P[1]) * x + P[0];
  d = ((4 * P[4] * x + 3 * P[3]) * x + 2 * P[2]) * x + P[1];
}

int main() {
  std::mt19937_64 g(2402);
  std::uniform_real_distribution<double> U(-1, 1);
  const double dlt = std::sqrt(3.0) / 6.0, xg[2] = {-0.5 - dlt, -0.5 + dlt};
  double e_gauss = 0, e_mean = 0, e_edge = 0, e_ind = 0, e_quad = 0;
  for (int it = 0; it < 200000; ++it) {
    const bool df = it % 3 == 0;
    const Coef<double> k = coef(df ? 0.5 : 0.0);
    const double ac = df ? 0.4 * (0.5 + 0.5 * U(g)) : 1.0;
    double Q[5];
    const double sc = std::pow(10.0, 3 * U(g));
    for (int m = 0; m < 5; ++m) Q[m] = 1 + sc * U(g);
    if (it % 4 == 1) for (int m = 0; m < 5; ++m) Q[m] = 2 + sc * std::sin(0.4 * m * U(g));
    if (it % 4 == 2) for (int m = 0; m < 5; ++m) Q[m] = m < it % 5 ? 1.0 : 1.0 + sc;
    double qa = 0;
    for (int m = 0; m < 5; ++m) qa = std::fmax(qa, std::fabs(Q[m]));
    double P[5], P2[2], v[2], d[2];
    recon_poly<double, 5>(Q, 0.1, ac, 0.2, k, P);
    recon_poly<double, 2>(Q, 0.1, ac, 0.2, k, P2);
    recon_gauss<double>(Q, 0.1, ac, 0.2, k, v, d);
    for (int q = 0; q < 2; ++q) {
      double pv, pd;
      poly_at(P, xg[q], pv, pd);
      e_gauss = std::fmax(e_gauss, std::fmax(std::fabs(pv - v[q]), std::fabs(pd - d[q])) / qa);
    }
    const double mean = P[0] - P[1] / 2 + P[2] / 3 - P[3] / 4 + P[4] / 5;
    e_mean = std::fmax(e_mean, std::fabs(mean - Q[2]) / qa);
    e_edge = std::fmax(e_edge, std::fmax(std::fabs(P2[0] - P[0]), std::fabs(P2[1] - P[1])) / qa);
    // Jiang-Shu: beta = (p'(centre))^2 + 13/12 (p'')^2 for quadratics in units of the cell width
    const WenoTerms<double> T = weno_terms(Q);
    const double a0 = Q[0] - 4 * Q[1] + 3 * Q[2], a1 = Q[3] - Q[1], a2 = -3 * Q[2] + 4 * Q[3] - Q[4];
    const double c0 = Q[0] - 2 * Q[1] + Q[2], c1 = Q[1] - 2 * Q[2] + Q[3], c2 = Q[2] - 2 * Q[3] + Q[4];
    const double bj[3] = {0.25 * a0 * a0 + 13.0 / 12.0 * c0 * c0, 0.25 * a1 * a1 + 13.0 / 12.0 * c1 * c1,
                          0.25 * a2 * a2 + 13.0 / 12.0 * c2 * c2};
    for (int q = 0; q < 3; ++q) e_ind = std::fmax(e_ind, std::fabs(T.b[q] - bj[q]) / (qa * qa));
    // cell averages of q(x) = A + B x + C x^2 over cells [m - 3, m - 2] (the target cell is [-1, 0])
    {
      const double A = U(g), B = U(g), C = U(g);
      double Qq[5];
      for (int m = 0; m < 5; ++m) {
        const double lo = m - 3.0, hi = m - 2.0;
        Qq[m] = A + B * (hi * hi - lo * lo) / 2 + C * (hi * hi * hi - lo * lo * lo) / 3;
      }
      const Coef<double> kw = coef(0.0);
      double Pq[2], vq[2], dq[2];
      recon_poly<double, 2>(Qq, 1.0, 1.0, 1.0, kw, Pq);
      recon_gauss<double>(Qq, 1.0, 1.0, 1.0, kw, vq, dq);
      double s = 1;
      for (int m = 0; m < 5; ++m) s = std::fmax(s, std::fabs(Qq[m]));
      e_quad = std::fmax(e_quad, std::fmax(std::fabs(Pq[0] - A), std::fabs(Pq[1] - B)) / s);
      for (int q = 0; q < 2; ++q) {
        const double x = xg[q];
        e_quad = std::fmax(e_quad, std::fmax(std::fabs(vq[q] - (A + B * x + C * x * x)),
                                             std::fabs(dq[q] - (B + 2 * C * x))) / s);
      }
    }
  }
  std::printf("gauss_vs_poly %.3e\ncell_mean %.3e\nedge_vs_poly %.3e\nindicators %.3e\nquadratic %.3e\n", e_gauss,
              e_mean, e_edge, e_ind, e_quad);
  return 0;
}
