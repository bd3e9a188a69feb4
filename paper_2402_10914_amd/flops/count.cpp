// Exact operation count of the HIP formulation: instantiates the kernels' own __host__ __device__
// arithmetic (dfw_math.hpp) on the host with a scalar that counts every add, multiply, divide,
// square root, exponential and erfc.  Counting convention: each of these is one flop (a fused
// multiply-add counts as its multiply and its add); comparisons, absolute values and negations
// are not counted.  Operations the compiler evaluates itself are not counted either: the scalar
// knows which values are constants of the source (literals and arithmetic on literals only), so an
// operation on two constants, and a multiplication or division by the constant 1 (or -1, a
// negation), count nothing, as on the GPU, where they never execute.  Inputs (states, scheme
// coefficients, time step) are run-time values.  The data is smooth (WENO-AO branch everywhere),
// the common path; the DF branch is cheaper.  Prints JSON.
#include <cmath>
#include <cstdio>

#include "../csrc/dfw_math.hpp"

namespace cnt {
long long n_add = 0, n_mul = 0, n_div = 0, n_sqrt = 0, n_exp = 0, n_erfc = 0;
struct C {
  double v;
  bool lit;  // a constant of the source
  C() : v(0), lit(true) {}
  C(double x) : v(x), lit(true) {}
  C(int x) : v(x), lit(true) {}
};
inline C value(double x, bool lit) {
  C c(x);
  c.lit = lit;
  return c;
}
inline C run(double x) { return value(x, false); }  // a run-time input
inline bool is(C a, double x) { return a.lit && a.v == x; }
inline C operator-(C a) { return value(-a.v, a.lit); }
inline C operator+(C a, C b) {
  if (a.lit && b.lit) return value(a.v + b.v, true);
  ++n_add;
  return run(a.v + b.v);
}
inline C operator-(C a, C b) {
  if (a.lit && b.lit) return value(a.v - b.v, true);
  ++n_add;
  return run(a.v - b.v);
}
inline C operator*(C a, C b) {
  if (a.lit && b.lit) return value(a.v * b.v, true);
  if (is(a, 1.0)) return b;
  if (is(b, 1.0)) return a;
  if (is(a, -1.0)) return -b;
  if (is(b, -1.0)) return -a;
  ++n_mul;
  return run(a.v * b.v);
}
inline C operator/(C a, C b) {
  if (a.lit && b.lit) return value(a.v / b.v, true);
  if (is(b, 1.0)) return a;
  ++n_div;
  return run(a.v / b.v);
}
inline C& operator+=(C& a, C b) { a = a + b; return a; }
inline C& operator*=(C& a, C b) { a = a * b; return a; }
inline bool operator<(C a, C b) { return a.v < b.v; }
inline bool operator>(C a, C b) { return a.v > b.v; }
inline bool operator>=(C a, C b) { return a.v >= b.v; }
inline C sqrt(C a) { if (a.lit) return value(std::sqrt(a.v), true); ++n_sqrt; return run(std::sqrt(a.v)); }
inline C exp(C a) { if (a.lit) return value(std::exp(a.v), true); ++n_exp; return run(std::exp(a.v)); }
inline C erfc(C a) { if (a.lit) return value(std::erfc(a.v), true); ++n_erfc; return run(std::erfc(a.v)); }
inline C fabs(C a) { return value(std::fabs(a.v), a.lit); }
long long total() { return n_add + n_mul + n_div + n_sqrt + n_exp + n_erfc; }
void reset() { n_add = n_mul = n_div = n_sqrt = n_exp = n_erfc = 0; }
}  // namespace cnt

using cnt::C;

static dfw::Coef<C> coef() {
  using cnt::run;
  dfw::Coef<C> k;
  double g = 1.4, dh = 0.85, dl = 0.85;
  k.gamma = run(g); k.gm1 = run(g - 1); k.inv_gm1 = run(1 / (g - 1)); k.alpha_thres = run(0.5); k.eps = run(1e-6);
  k.c1 = run(0.01); k.c2 = run(5.0); k.K = run((4 - 2 * g) / (g - 1));
  double d[4] = {(1 - dh) * (1 - dl) / 2, (1 - dh) * dl, (1 - dh) * (1 - dl) / 2, dh};
  for (int i = 0; i < 4; ++i) k.d[i] = run(d[i]);
  for (int i = 0; i < 3; ++i) k.dr[i] = run(d[i] / d[3]);
  k.inv_d3 = run(1 / d[3]);
  k.K2 = run(k.K.v + 2); k.k4K2 = run(4 / (k.K.v + 2));
  k.sw_rule = 0;
  return k;
}

static void state(double x, C* w) {  // smooth sample state
  double r = 1 + 0.2 * std::sin(x), u = 0.3 + 0.1 * std::cos(x), v = -0.2 + 0.1 * std::sin(2 * x), p = 1 + 0.1 * std::cos(x);
  w[0] = cnt::run(r); w[1] = cnt::run(r * u); w[2] = cnt::run(r * v);
  w[3] = cnt::run(p / 0.4 + 0.5 * r * (u * u + v * v));
}

struct Count { long long total, div, sqrt_, exp_, erfc_; };
static Count snap() { return Count{cnt::total(), cnt::n_div, cnt::n_sqrt, cnt::n_exp, cnt::n_erfc}; }

template <int FLUX, bool F, bool DF>
static Count segment() {
  dfw::Coef<C> k = coef();
  C wa[4], wb[4], wln[4], wrn[4], lines[2][5][4];
  state(0.1, wa); state(0.2, wb); state(0.3, wln); state(0.4, wrn);
  for (int s = 0; s < 2; ++s) for (int m = 0; m < 5; ++m) state(0.05 * (m + 3 * s), lines[s][m]);
  for (int c = 0; c < 4; ++c) { wln[c] = wln[c] * C(0.01); wrn[c] = wrn[c] * C(0.01); }
  C al[2][3];
  for (int s = 0; s < 2; ++s) for (int q = 0; q < 3; ++q) al[s][q] = cnt::run(1.0);
  auto line = [&](int side, int m, int c) -> C { return lines[side][m][c]; };
  C Fs[4], Fts[4], dfp;
  cnt::reset();
  dfw::segment_fluxes<C, FLUX, F, DF>(wa, wb, line, al, wln, wrn, cnt::run(1e-3), cnt::run(100.0), k, Fs, Fts, dfp);
  return snap();
}

static Count normal() {
  dfw::Coef<C> k = coef();
  C cell[6][4], wl[4], wr[4], wln[4], wrn[4];
  for (int m = 0; m < 6; ++m) state(0.05 * m, cell[m]);
  cnt::reset();
  const C one = cnt::run(1.0);
  dfw::normal_sweep<C>(cell, one, one, one, one, cnt::run(100.0), k, wl, wr, wln, wrn);
  return snap();
}

static void print(const char* name, Count c, bool comma) {
  std::printf("  \"%s\": {\"flops\": %lld, \"div\": %lld, \"sqrt\": %lld, \"exp\": %lld, \"erfc\": %lld}%s\n", name,
              c.total, c.div, c.sqrt_, c.exp_, c.erfc_, comma ? "," : "");
}

int main() {
  // Cell kernels (per cell): update 1 forms L and dL/dt from four face sums (16 sub, 16 mul,
  // 8 add) and W*, R (3 coefficient products, 16 mul, 16 add); update 2 forms dL/dt (20), the new
  // state (1 + 8), the DF product (3) and the signal speed (1 div, 8 mul/add, 1 sqrt, 2 mul).
  std::printf("{\n");
  print("normal_sweep", normal(), true);
  print("segment_lf_stage1", segment<0, true, false>(), true);
  print("segment_lf_stage2", segment<0, false, true>(), true);
  print("segment_gks_stage1", segment<1, true, false>(), true);
  print("segment_gks_stage2", segment<1, false, true>(), true);
  std::printf("  \"update1_per_cell\": 75,\n  \"update2_per_cell\": 45\n}\n");
  return 0;
}
