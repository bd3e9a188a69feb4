// Exact operation count of the HIP formulation: instantiates the kernels' own __host__ __device__
// arithmetic (dfw_math.hpp) on the host with a scalar that counts every add, multiply, divide,
// square root, exponential and erfc.  Counting convention: each of these is one flop (a fused
// multiply-add counts as its multiply and its add); comparisons, absolute values and negations
// are not counted.  The data is smooth (WENO-AO branch everywhere), the common path; the DF branch
// is cheaper.  Prints JSON.
#include <cmath>
#include <cstdio>

#include "../csrc/dfw_math.hpp"

namespace cnt {
long long n_add = 0, n_mul = 0, n_div = 0, n_sqrt = 0, n_exp = 0, n_erfc = 0;
struct C {
  double v;
  C() : v(0) {}
  C(double x) : v(x) {}
  C(int x) : v(x) {}
};
inline C operator+(C a, C b) { ++n_add; return C(a.v + b.v); }
inline C operator-(C a, C b) { ++n_add; return C(a.v - b.v); }
inline C operator*(C a, C b) { ++n_mul; return C(a.v * b.v); }
inline C operator/(C a, C b) { ++n_div; return C(a.v / b.v); }
inline C operator-(C a) { return C(-a.v); }
inline C& operator+=(C& a, C b) { a = a + b; return a; }
inline C& operator*=(C& a, C b) { a = a * b; return a; }
inline bool operator<(C a, C b) { return a.v < b.v; }
inline bool operator>(C a, C b) { return a.v > b.v; }
inline bool operator>=(C a, C b) { return a.v >= b.v; }
inline C sqrt(C a) { ++n_sqrt; return C(std::sqrt(a.v)); }
inline C exp(C a) { ++n_exp; return C(std::exp(a.v)); }
inline C erfc(C a) { ++n_erfc; return C(std::erfc(a.v)); }
inline C fabs(C a) { return C(std::fabs(a.v)); }
long long total() { return n_add + n_mul + n_div + n_sqrt + n_exp + n_erfc; }
void reset() { n_add = n_mul = n_div = n_sqrt = n_exp = n_erfc = 0; }
}  // namespace cnt

using cnt::C;

static dfw::Coef<C> coef() {
  dfw::Coef<C> k;
  double g = 1.4, dh = 0.85, dl = 0.85;
  k.gamma = g; k.gm1 = g - 1; k.inv_gm1 = 1 / (g - 1); k.alpha_thres = 0.5; k.eps = 1e-6;
  k.c1 = 0.01; k.c2 = 5.0; k.K = (4 - 2 * g) / (g - 1);
  double d[4] = {(1 - dh) * (1 - dl) / 2, (1 - dh) * dl, (1 - dh) * (1 - dl) / 2, dh};
  for (int i = 0; i < 4; ++i) k.d[i] = d[i];
  for (int i = 0; i < 3; ++i) k.dr[i] = d[i] / d[3];
  k.inv_d3 = 1 / d[3];
  k.K2 = k.K.v + 2; k.k4K2 = 4 / (k.K.v + 2);
  k.sw_rule = 0;
  return k;
}

static void state(double x, C* w) {  // smooth sample state
  double r = 1 + 0.2 * std::sin(x), u = 0.3 + 0.1 * std::cos(x), v = -0.2 + 0.1 * std::sin(2 * x), p = 1 + 0.1 * std::cos(x);
  w[0] = r; w[1] = r * u; w[2] = r * v; w[3] = p / 0.4 + 0.5 * r * (u * u + v * v);
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
  for (int s = 0; s < 2; ++s) for (int q = 0; q < 3; ++q) al[s][q] = 1.0;
  auto line = [&](int side, int m, int c) -> C { return lines[side][m][c]; };
  C Fs[4], Fts[4], dfp;
  cnt::reset();
  dfw::segment_fluxes<C, FLUX, F, DF>(wa, wb, line, al, wln, wrn, C(1e-3), C(100.0), k, Fs, Fts, dfp);
  return snap();
}

static Count normal() {
  dfw::Coef<C> k = coef();
  C cell[6][4], wl[4], wr[4], wln[4], wrn[4];
  for (int m = 0; m < 6; ++m) state(0.05 * m, cell[m]);
  cnt::reset();
  dfw::normal_sweep<C>(cell, C(1.0), C(1.0), C(1.0), C(1.0), C(100.0), k, wl, wr, wln, wrn);
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
