// Host-side check of the hand-written adjoints in dfw_adjoint.hpp: for random inputs x, random
// output seeds l and random directions v, the adjoint's <adj(l), v> must equal the central
// difference <l, (f(x + h v) - f(x - h v)) / 2h> of the forward device function.  Prints one line
// per check: name, relative difference.  Built and run by tests/test_adjoint_local.py.
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

#include "../paper_2402_10914_amd/csrc/dfw_adjoint.hpp"

using namespace dfw;
using real = double;

static Coef<real> coef(double alpha_thres = 0.5, double c1 = 0.01, double c2 = 5.0) {
  Coef<real> k;
  double g = 1.4, dh = 0.85, dl = 0.85;
  k.gamma = g;
  k.gm1 = g - 1;
  k.inv_gm1 = 1 / (g - 1);
  k.alpha_thres = alpha_thres;
  k.eps = 1e-6;
  k.c1 = c1;
  k.c2 = c2;
  k.K = (4 - 2 * g) / (g - 1);
  double d[4] = {(1 - dh) * (1 - dl) / 2, (1 - dh) * dl, (1 - dh) * (1 - dl) / 2, dh};
  for (int i = 0; i < 4; ++i) k.d[i] = d[i];
  for (int i = 0; i < 3; ++i) k.dr[i] = d[i] / d[3];
  k.inv_d3 = 1 / d[3];
  k.K2 = k.K + 2;
  k.k4K2 = 4 / (k.K + 2);
  k.sw_rule = 0;
  return k;
}

static std::mt19937_64 rng(12345);
static double unif(double a, double b) { return std::uniform_real_distribution<double>(a, b)(rng); }

static void rand_state(real* w, double jitter = 1.0) {
  double r = unif(0.5, 1.5), u = unif(-0.8, 0.8) * jitter, v = unif(-0.8, 0.8) * jitter, p = unif(0.5, 1.5);
  w[0] = r;
  w[1] = r * u;
  w[2] = r * v;
  w[3] = p / 0.4 + 0.5 * r * (u * u + v * v);
}

// Generic check: x (n inputs), f: x -> y (m outputs), adj: (x, ly) -> lx.
template <class F, class A>
static double check(const char* name, std::vector<double> x, int m, F f, A adj, double h = 1e-6) {
  const int n = (int)x.size();
  std::vector<double> l(m), v(n), lx(n, 0.0), yp(m), ym(m), xp(n), xm(n);
  for (auto& e : l) e = unif(-1, 1);
  for (int i = 0; i < n; ++i) v[i] = unif(-1, 1) * (std::fabs(x[i]) + 0.1);
  for (int i = 0; i < n; ++i) {
    xp[i] = x[i] + h * v[i];
    xm[i] = x[i] - h * v[i];
  }
  f(xp.data(), yp.data());
  f(xm.data(), ym.data());
  double fd = 0;
  for (int j = 0; j < m; ++j) fd += l[j] * (yp[j] - ym[j]) / (2 * h);
  adj(x.data(), l.data(), lx.data());
  double ad = 0;
  for (int i = 0; i < n; ++i) ad += lx[i] * v[i];
  double rel = std::fabs(fd - ad) / std::max(std::fabs(fd), 1e-12);
  std::printf("%s %.3e fd %.10e adj %.10e\n", name, rel, fd, ad);
  return rel;
}

int main() {
  Coef<real> k = coef();
  for (int trial = 0; trial < 3; ++trial) {
    // ---- basis + project + unproject
    {
      std::vector<double> x(12);
      rand_state(&x[0]);
      rand_state(&x[4]);
      rand_state(&x[8]);
      check("project", x, 4,
            [&](const double* xx, double* y) {
              Basis<real> B = make_basis(xx, xx + 4, k);
              project(B, xx + 8, y);
            },
            [&](const double* xx, const double* l, double* lx) {
              Basis<real> B = make_basis(xx, xx + 4, k);
              BasisAdj<real> lB;
              lB.zero();
              project_adj(B, xx + 8, l, lx + 8, lB);
              make_basis_adj(xx, xx + 4, k, lB, lx, lx + 4);
            });
      check("unproject", x, 4,
            [&](const double* xx, double* y) {
              Basis<real> B = make_basis(xx, xx + 4, k);
              unproject(B, xx + 8, y);
            },
            [&](const double* xx, const double* l, double* lx) {
              Basis<real> B = make_basis(xx, xx + 4, k);
              BasisAdj<real> lB;
              lB.zero();
              unproject_adj(B, xx + 8, l, lx + 8, lB);
              make_basis_adj(xx, xx + 4, k, lB, lx, lx + 4);
            });
    }
    // ---- reconstruction, both branches
    for (int branch = 0; branch < 2; ++branch) {
      std::vector<double> x(6);
      for (int i = 0; i < 5; ++i) x[i] = 1.0 + 0.3 * std::sin(0.7 * i + trial) + unif(-0.2, 0.2);
      x[5] = branch ? 0.3 : 0.9;  // centre alpha
      double alo = branch ? 0.2 : 0.8, ahi = branch ? 0.1 : 0.95;
      auto f5 = [&](const double* xx, double* y) {
        real P[5];
        recon_poly<real, 5>(xx, alo, xx[5], ahi, k, P);
        for (int i = 0; i < 5; ++i) y[i] = P[i];
      };
      auto a5 = [&](const double* xx, const double* l, double* lx) {
        recon_poly_adj<real, 5>(xx, alo, xx[5], ahi, k, l, lx, lx[5]);
      };
      check(branch ? "recon5_df" : "recon5_weno", x, 5, f5, a5);
      auto f2 = [&](const double* xx, double* y) {
        real P[2];
        recon_poly<real, 2>(xx, alo, xx[5], ahi, k, P);
        y[0] = P[0];
        y[1] = P[1];
      };
      auto a2 = [&](const double* xx, const double* l, double* lx) {
        recon_poly_adj<real, 2>(xx, alo, xx[5], ahi, k, l, lx, lx[5]);
      };
      check(branch ? "recon2_df" : "recon2_weno", x, 2, f2, a2);
      auto fg = [&](const double* xx, double* y) {
        real v[2], d[2];
        recon_gauss<real>(xx, alo, xx[5], ahi, k, v, d);
        y[0] = v[0];
        y[1] = v[1];
        y[2] = d[0];
        y[3] = d[1];
      };
      auto ag = [&](const double* xx, const double* l, double* lx) {
        real v[2], d[2];
        recon_gauss_adj<real>(xx, alo, xx[5], ahi, k, l, l + 2, lx, lx[5], v, d);
      };
      check(branch ? "recon_gauss_df" : "recon_gauss_weno", x, 4, fg, ag);
    }
    // ---- prim + DF
    {
      std::vector<double> x(8);
      rand_state(&x[0]);
      rand_state(&x[4]);
      check("df_factor", x, 1,
            [&](const double* xx, double* y) { y[0] = df_factor(prim(xx, k), prim(xx + 4, k)); },
            [&](const double* xx, const double* l, double* lx) {
              Prim<real> L = prim(xx, k), R = prim(xx + 4, k);
              PrimAdj<real> lL, lR;
              lL.zero();
              lR.zero();
              df_factor_adj(L, R, l[0], lL, lR);
              prim_adj(xx, L, k, lL, lx);
              prim_adj(xx + 4, R, k, lR, lx + 4);
            });
    }
    // ---- fluxes: inputs wl, wln, wlt, wr, wrn, wrt (24); outputs F, Ft (8)
    for (int flux = 0; flux < 2; ++flux) {
      for (int taumode = 0; taumode < (flux ? 2 : 1); ++taumode) {
        Coef<real> kk = taumode ? coef(0.5, 0.0, 0.0) : k;
        std::vector<double> x(24);
        rand_state(&x[0]);
        rand_state(&x[12]);
        for (int i = 0; i < 4; ++i) {
          x[4 + i] = unif(-0.5, 0.5);
          x[8 + i] = unif(-0.5, 0.5);
          x[16 + i] = unif(-0.5, 0.5);
          x[20 + i] = unif(-0.5, 0.5);
        }
        const real dt = 2e-3;
        auto f = [&](const double* xx, double* y) {
          Prim<real> ql = prim(xx, kk), qr = prim(xx + 12, kk);
          if (flux == 0) lf_flux<real, true>(xx, xx + 4, xx + 8, xx + 12, xx + 16, xx + 20, ql, qr, kk, y, y + 4);
          else gks_flux<real, true>(xx, xx + 4, xx + 8, xx + 12, xx + 16, xx + 20, ql, qr, dt, kk, y, y + 4);
        };
        auto a = [&](const double* xx, const double* l, double* lx) {
          Prim<real> ql = prim(xx, kk), qr = prim(xx + 12, kk);
          PrimAdj<real> lql, lqr;
          lql.zero();
          lqr.zero();
          if (flux == 0)
            lf_flux_adj(xx, xx + 4, xx + 8, xx + 12, xx + 16, xx + 20, ql, qr, kk, l, l + 4, lx, lx + 4, lx + 8,
                        lx + 12, lx + 16, lx + 20, lql, lqr);
          else
            gks_flux_adj(xx, xx + 4, xx + 8, xx + 12, xx + 16, xx + 20, ql, qr, dt, kk, l, l + 4, lx, lx + 4, lx + 8,
                         lx + 12, lx + 16, lx + 20, lql, lqr);
          prim_adj(xx, ql, kk, lql, lx);
          prim_adj(xx + 12, qr, kk, lqr, lx + 12);
        };
        check(flux ? (taumode ? "gks_flux_tau0" : "gks_flux") : "lf_flux", x, 8, f, a);
      }
    }
    // ---- normal sweep: 6 cells (24) + 4 alphas -> wl, wr, wln, wrn (16).  The adjoint is composed
    //      from the two one-side pieces and the basis adjoint, as the interface kernel composes it.
    for (int branch = 0; branch < 2; ++branch) {
      std::vector<double> x(28);
      for (int m = 0; m < 6; ++m) rand_state(&x[4 * m], 0.5);
      for (int i = 0; i < 4; ++i) x[24 + i] = branch ? 0.3 : 1.0;
      const real idn = 50.0;
      auto f = [&](const double* xx, double* y) {
        real cell[6][4];
        for (int m = 0; m < 6; ++m)
          for (int c = 0; c < 4; ++c) cell[m][c] = xx[4 * m + c];
        normal_sweep<real>(cell, xx[24], xx[25], xx[26], xx[27], idn, k, y, y + 4, y + 8, y + 12);
      };
      auto a = [&](const double* xx, const double* l, double* lx) {
        real cs0[5][4], cs1[5][4], lcs0[5][4] = {}, lcs1[5][4] = {};
        for (int m = 0; m < 5; ++m)
          for (int c = 0; c < 4; ++c) {
            cs0[m][c] = xx[4 * m + c];
            cs1[m][c] = xx[4 * (5 - m) + c];
          }
        Basis<real> B = make_basis(xx + 8, xx + 12, k);
        BasisAdj<real> lB;
        lB.zero();
        real la1 = 0, la2 = 0;
        auto c0 = [&](int m, int c) -> real { return cs0[m][c]; };
        auto c1 = [&](int m, int c) -> real { return cs1[m][c]; };
        auto add0 = [&](int m, int c, real v) { lcs0[m][c] += v; };
        auto add1 = [&](int m, int c, real v) { lcs1[m][c] += v; };
        normal_side_adj(B, c0, xx[24], xx[25], xx[26], idn, k, l, l + 8, add0, lB, la1);
        normal_side_adj(B, c1, xx[27], xx[26], xx[25], -idn, k, l + 4, l + 12, add1, lB, la2);
        for (int m = 0; m < 5; ++m)
          for (int c = 0; c < 4; ++c) {
            lx[4 * m + c] += lcs0[m][c];
            lx[4 * (5 - m) + c] += lcs1[m][c];
          }
        make_basis_adj(xx + 8, xx + 12, k, lB, lx + 8, lx + 12);
        lx[25] += la1;
        lx[26] += la2;
      };
      check(branch ? "normal_sweep_df" : "normal_sweep", x, 16, f, a);
      // the one-side forward pieces reproduce the whole sweep
      {
        real y[16], cell[6][4], cs0[5][4], cs1[5][4], w[16];
        for (int m = 0; m < 6; ++m)
          for (int c = 0; c < 4; ++c) cell[m][c] = x[4 * m + c];
        for (int m = 0; m < 5; ++m)
          for (int c = 0; c < 4; ++c) {
            cs0[m][c] = cell[m][c];
            cs1[m][c] = cell[5 - m][c];
          }
        normal_sweep<real>(cell, x[24], x[25], x[26], x[27], idn, k, y, y + 4, y + 8, y + 12);
        Basis<real> B = make_basis(cell[2], cell[3], k);
        normal_side(B, cs0, x[24], x[25], x[26], idn, k, w, w + 8);
        normal_side(B, cs1, x[27], x[26], x[25], -idn, k, w + 4, w + 12);
        double d = 0;
        for (int i = 0; i < 16; ++i) d = std::max(d, std::fabs(w[i] - y[i]) / (std::fabs(y[i]) + 1e-300));
        std::printf("%s %.3e\n", branch ? "normal_side_fwd_df" : "normal_side_fwd", d);
      }
    }
    // ---- segment: wa, wb (8), lines 2x5x4 (40), wln, wrn (8), centre alphas (2) -> Fs, Fts, dfp (9).
    //      Adjoint composed from the one-side pieces, the per-Gauss-point flux adjoint and the basis
    //      adjoint, as the interface kernel composes it.
    for (int flux = 0; flux < 2; ++flux)
      for (int branch = 0; branch < 2; ++branch) {
        std::vector<double> x(58);
        rand_state(&x[0], 0.5);
        rand_state(&x[4], 0.5);
        for (int s = 0; s < 2; ++s)
          for (int m = 0; m < 5; ++m) rand_state(&x[8 + 20 * s + 4 * m], 0.5);
        for (int i = 0; i < 8; ++i) x[48 + i] = unif(-0.3, 0.3);
        x[56] = branch ? 0.3 : 1.0;
        x[57] = branch ? 0.2 : 1.0;
        const real dt = 2e-3, idt = 40.0;
        auto alphas = [&](const double* xx, real (*al)[3]) {
          const real a[2][3] = {{branch ? 0.1 : 1.0, xx[56], 0.2}, {0.3, xx[57], branch ? 0.4 : 1.0}};
          for (int s = 0; s < 2; ++s)
            for (int q = 0; q < 3; ++q) al[s][q] = a[s][q];
        };
        auto run = [&](const double* xx, double* y) {
          auto line = [&](int side, int m, int c) -> real { return xx[8 + 20 * side + 4 * m + c]; };
          real al[2][3];
          alphas(xx, al);
          real dfp;
          if (flux == 0) segment_fluxes<real, 0, true, true>(xx, xx + 4, line, al, xx + 48, xx + 52, dt, idt, k, y, y + 4, dfp);
          else segment_fluxes<real, 1, true, true>(xx, xx + 4, line, al, xx + 48, xx + 52, dt, idt, k, y, y + 4, dfp);
          y[8] = dfp;
        };
        auto a = [&](const double* xx, const double* l, double* lx) {
          real al[2][3];
          alphas(xx, al);
          Basis<real> B = make_basis(xx, xx + 4, k);
          real gw[2][2][4], gwt[2][2][4];
          for (int s = 0; s < 2; ++s) {
            auto line = [&](int m, int c) -> real { return xx[8 + 20 * s + 4 * m + c]; };
            segment_side(B, line, al[s], idt, k, gw[s], gwt[s]);
          }
          real dfg[2];
          for (int g = 0; g < 2; ++g) dfg[g] = df_factor(prim(gw[0][g], k), prim(gw[1][g], k));
          real lgw[2][2][4] = {}, lgwt[2][2][4] = {};
          for (int g = 0; g < 2; ++g) {
            if (flux == 0)
              gp_flux_adj<real, 0>(gw[0][g], xx + 48, gwt[0][g], gw[1][g], xx + 52, gwt[1][g], dt, k, l, l + 4,
                                   l[8] * dfg[1 - g], lgw[0][g], lx + 48, lgwt[0][g], lgw[1][g], lx + 52, lgwt[1][g]);
            else
              gp_flux_adj<real, 1>(gw[0][g], xx + 48, gwt[0][g], gw[1][g], xx + 52, gwt[1][g], dt, k, l, l + 4,
                                   l[8] * dfg[1 - g], lgw[0][g], lx + 48, lgwt[0][g], lgw[1][g], lx + 52, lgwt[1][g]);
          }
          BasisAdj<real> lB;
          lB.zero();
          real lac[2] = {0, 0};
          for (int s = 0; s < 2; ++s) {
            auto line = [&](int m, int c) -> real { return xx[8 + 20 * s + 4 * m + c]; };
            real ll[5][4] = {};
            auto add = [&](int m, int c, real v) { ll[m][c] += v; };
            segment_side_adj(B, line, al[s], idt, k, lgw[s], lgwt[s], add, lB, lac[s]);
            for (int m = 0; m < 5; ++m)
              for (int c = 0; c < 4; ++c) lx[8 + 20 * s + 4 * m + c] += ll[m][c];
          }
          make_basis_adj(xx, xx + 4, k, lB, lx, lx + 4);
          lx[56] += lac[0];
          lx[57] += lac[1];
        };
        const char* names[2][2] = {{"segment_lf", "segment_lf_df"}, {"segment_gks", "segment_gks_df"}};
        check(names[flux][branch], x, 9, run, a);
      }
  }
  return 0;
}
