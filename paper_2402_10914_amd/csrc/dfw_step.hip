// HIP kernels and C ABI of the S2O4 DF-hybrid step for gfx950 (Zhang, Ji & Xu, arXiv:2402.10914).
//
// One step = [faces(stage 1)] [update 1] [faces(stage 2)] [update 2]:
//   faces:   one launch covers every x- and y-interface.  A workgroup owns a tile of TF interfaces
//            (along the normal) by TR interface segments (along the tangential direction).  It
//            stages the (TF+5) x (TR+4) cells and the alpha halo in LDS once (ghost cells by index
//            mapping), runs the normal reconstruction for TR+4 segments per interface column into
//            LDS, then the tangential reconstruction at the two Gauss points of each of its TR
//            segments, the flux and its time derivative, and the DF of the Gauss points.  The
//            thread that reconstructs a segment in the normal sweep also owns it in the
//            tangential sweep, so the normal derivatives stay in registers.
//   update:  one thread per cell assembles L and dL/dt from the four face sums (eq. (2)) and
//            applies eq. (24); the second update also forms alpha^{n+1} (Section 3.2), checks
//            positivity and reduces the signal speed for the next dt (wavefront shuffle, LDS,
//            one 64-bit atomic max per workgroup on the bit pattern of a non-negative double).
// dt lives in device memory; the host never reads it inside a run.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/dfweno.h"
#include "dfw_math.hpp"

namespace dfw {

// ------------------------------------------------------------------------------------------------
// Device control block (in the workspace).
// ------------------------------------------------------------------------------------------------
struct Ctrl {
  unsigned long long smax_bits[2];  // running max signal speed / dx for the next step (ping-pong)
  double dt;                        // dt of the current step
  double t;                         // accumulated time
  int status;                       // 0 ok, 1 non-physical state met
  int fail_step;                    // completed steps when status was raised
  int pad[2];
};

struct KParams {
  int nx, ny, bc_x, bc_y;
  double dx, dy, inv_dx, inv_dy;
  double gamma, cfl, dt_fixed, alpha_thres, eps, c1, c2, K;
  double d[4];
};

enum { OUT_F = 1, OUT_FT = 2, OUT_DF = 4 };

template <class real>
__device__ __forceinline__ Coef<real> make_coef(const KParams& P) {
  Coef<real> k;
  k.gamma = real(P.gamma);
  k.gm1 = real(P.gamma - 1.0);
  k.inv_gm1 = real(1.0 / (P.gamma - 1.0));
  k.alpha_thres = real(P.alpha_thres);
  k.eps = real(P.eps);
  k.c1 = real(P.c1);
  k.c2 = real(P.c2);
  k.K = real(P.K);
  for (int i = 0; i < 4; ++i) k.d[i] = real(P.d[i]);
  for (int i = 0; i < 3; ++i) k.dr[i] = real(P.d[i] / P.d[3]);
  k.inv_d3 = real(1.0 / P.d[3]);
  return k;
}

__device__ __forceinline__ int bc_map(int i, int n, int bc) {
  if (bc == DFW_BC_PERIODIC) {
    int r = i % n;
    return r < 0 ? r + n : r;
  }
  return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

// ------------------------------------------------------------------------------------------------
// Face kernel.
// Face arrays: FX [9][ny][nx+1] and FY [9][ny+1][nx]; entries 0..3 = face-averaged flux (global
// components), 4..7 = its time derivative, 8 = product of the DF of the two Gauss points.
// ------------------------------------------------------------------------------------------------
template <int TF, int TR>
struct Tile {
  static constexpr int NR = TR + 4;         // segments incl. the normal-sweep halo
  static constexpr int NT = TF * NR;        // threads per workgroup
  static constexpr int WN = TF + 5;         // cells along the normal
  static constexpr int AN = TF + 3;         // alpha cells along the normal
};

template <class real, int FLUX, int OUT, int TF, int TR>
__global__ __launch_bounds__(TF * (TR + 4)) void k_faces(const real* __restrict__ W,
                                                              const real* __restrict__ alpha,
                                                              real* __restrict__ FX, real* __restrict__ FY,
                                                              Ctrl* __restrict__ ctrl, KParams P, double dt_host,
                                                              int lead, int step, double* __restrict__ dt_hist) {
  using T = Tile<TF, TR>;
  if (ctrl->status) return;
  __shared__ real sW[4][T::NR][T::WN];
  __shared__ real sA[T::NR][T::AN];
  __shared__ real sLine[8][T::NT];

  const int nx = P.nx, ny = P.ny;
  // ---- which tile: x-interfaces first, then y-interfaces
  const int ntfx = (nx + 1 + TF - 1) / TF, ntrx = (ny + TR - 1) / TR;
  const int nbx = ntfx * ntrx;
  int b = blockIdx.x;
  const int dir = b < nbx ? 0 : 1;
  if (dir) b -= nbx;
  const int Nn = dir ? ny : nx, Nt = dir ? nx : ny;
  const int ntf = dir ? (ny + 1 + TF - 1) / TF : ntfx;
  const int f0 = (b % ntf) * TF, t0 = (b / ntf) * TR;
  const int bcn = dir ? P.bc_y : P.bc_x, bct = dir ? P.bc_x : P.bc_y;
  const real inv_dn = real(dir ? P.inv_dy : P.inv_dx), inv_dt = real(dir ? P.inv_dx : P.inv_dy);
  const size_t N = (size_t)nx * ny;
  const int tid = threadIdx.x;

  // ---- dt of this step
  double dtd;
  if (dt_host > 0.0) dtd = dt_host;
  else if (lead) dtd = P.cfl / __longlong_as_double((long long)ctrl->smax_bits[step & 1]);
  else dtd = ctrl->dt;
  if (lead && blockIdx.x == 0 && tid == 0) {
    ctrl->dt = dtd;
    ctrl->t += dtd;
    ctrl->smax_bits[(step + 1) & 1] = 0ull;
    if (dt_hist) dt_hist[step] = dtd;
  }
  const real dt = real(dtd);
  const Coef<real> k = make_coef<real>(P);

  // ---- stage cells and alpha into LDS (ghost cells by index mapping); component order local:
  //      0 rho, 1 normal momentum, 2 tangential momentum, 3 energy
  for (int e = tid; e < T::NR * T::WN; e += T::NT) {
    int nl, tl;
    if (dir == 0) { tl = e / T::WN; nl = e % T::WN; }
    else { nl = e / T::NR; tl = e % T::NR; }
    int n = bc_map(f0 - 3 + nl, Nn, bcn), t = bc_map(t0 - 2 + tl, Nt, bct);
    size_t g = dir == 0 ? (size_t)t * nx + n : (size_t)n * nx + t;
    sW[0][tl][nl] = W[g];
    sW[1][tl][nl] = W[(dir ? 2 : 1) * N + g];
    sW[2][tl][nl] = W[(dir ? 1 : 2) * N + g];
    sW[3][tl][nl] = W[3 * N + g];
  }
  for (int e = tid; e < T::NR * T::AN; e += T::NT) {
    int nl, tl;
    if (dir == 0) { tl = e / T::AN; nl = e % T::AN; }
    else { nl = e / T::NR; tl = e % T::NR; }
    int n = bc_map(f0 - 2 + nl, Nn, bcn), t = bc_map(t0 - 2 + tl, Nt, bct);
    size_t g = dir == 0 ? (size_t)t * nx + n : (size_t)n * nx + t;
    sA[tl][nl] = alpha[g];
  }
  __syncthreads();

  // ---- item owned by this thread: interface column fl, segment row rr (row t = t0 - 2 + rr)
  int fl, rr;
  if (dir == 0) { fl = tid % TF; rr = tid / TF; }
  else { rr = tid % T::NR; fl = tid / T::NR; }
  const int rstride = dir == 0 ? TF : 1;  // thread-index distance between neighbouring rows
  const int f = f0 + fl, t = t0 - 2 + rr;
  const bool live1 = f <= Nn && t < Nt + 2;
  real wln[4] = {0, 0, 0, 0}, wrn[4] = {0, 0, 0, 0};

  // ---- normal sweep (Section 3.1): line values of both sides and their normal derivatives
  if (live1) {
    real cell[6][4];
#pragma unroll
    for (int m = 0; m < 6; ++m)
#pragma unroll
      for (int c = 0; c < 4; ++c) cell[m][c] = sW[c][rr][fl + m];
    real wl[4], wr[4];
    normal_sweep<real>(cell, sA[rr][fl], sA[rr][fl + 1], sA[rr][fl + 2], sA[rr][fl + 3], inv_dn, k, wl, wr, wln, wrn);
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
  segment_fluxes<real, FLUX, (OUT & OUT_F) != 0, (OUT & OUT_DF) != 0>(wa, wb, line, al, wln, wrn, dt, inv_dt, k, Fs,
                                                                        Fts, dfp);
  // ---- write face sums (quadrature weights 1/2), components back to the global order
  const size_t fstride = dir == 0 ? (size_t)ny * (nx + 1) : (size_t)(ny + 1) * nx;
  real* Fo = dir == 0 ? FX + (size_t)t * (nx + 1) + f : FY + (size_t)f * nx + t;
  const int cmap[4] = {0, dir ? 2 : 1, dir ? 1 : 2, 3};
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    if (OUT & OUT_F) Fo[cmap[c] * fstride] = real(0.5) * Fs[c];
    if (OUT & OUT_FT) Fo[(4 + cmap[c]) * fstride] = real(0.5) * Fts[c];
  }
  if (OUT & OUT_DF) Fo[8 * fstride] = dfp;
}

// ------------------------------------------------------------------------------------------------
// Cell kernels.
// ------------------------------------------------------------------------------------------------
template <class real>
__device__ __forceinline__ void face_sum(const real* FX, const real* FY, const KParams& P, int i, int j, int base,
                                         real* out) {
  // no contraction here: the x and y contributions are rounded alike, so a transposed grid
  // (x <-> y, U <-> V) gives a bitwise transposed result
#pragma clang fp contract(off)
  const int nx = P.nx, ny = P.ny;
  const size_t sx = (size_t)ny * (nx + 1), sy = (size_t)(ny + 1) * nx;
  const size_t w = (size_t)j * (nx + 1) + i, s = (size_t)j * nx + i;
  const real ix = real(P.inv_dx), iy = real(P.inv_dy);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const real* fx = FX + (base + c) * sx;
    const real* fy = FY + (base + c) * sy;
    real ax = (fx[w] - fx[w + 1]) * ix;
    real ay = (fy[s] - fy[s + nx]) * iy;
    out[c] = ax + ay;
  }
}

template <class real>
__global__ __launch_bounds__(256) void k_update1(const real* __restrict__ W, const real* __restrict__ FX,
                                                 const real* __restrict__ FY, real* __restrict__ Ws,
                                                 real* __restrict__ R, Ctrl* __restrict__ ctrl, KParams P) {
  if (ctrl->status) return;
  const size_t N = (size_t)P.nx * P.ny, o = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= N) return;
  const int i = (int)(o % P.nx), j = (int)(o / P.nx);
  const real dt = real(ctrl->dt);
  real L[4], Lt[4];
  face_sum(FX, FY, P, i, j, 0, L);
  face_sum(FX, FY, P, i, j, 4, Lt);
  const real h1 = real(0.5) * dt, h2 = dt * dt * real(0.125), r2 = dt * dt * real(1.0 / 6.0);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    real w = W[c * N + o];
    Ws[c * N + o] = w + h1 * L[c] + h2 * Lt[c];
    R[c * N + o] = w + dt * L[c] + r2 * Lt[c];
  }
}

template <class real>
__device__ __forceinline__ bool cell_speed(const real* w, const KParams& P, double& s) {
  const real g = real(P.gamma);
  real ir = real(1) / w[0];
  real u = w[1] * ir, v = w[2] * ir;
  real p = real(P.gamma - 1.0) * (w[3] - real(0.5) * (w[1] * u + w[2] * v));
  bool ok = w[0] > real(0) && p > real(0) && isfinite(w[1]) && isfinite(w[2]) && isfinite(w[3]) && isfinite(p);
  real c = sqrt(g * p * ir);
  real sx = (fabs(u) + c) * real(P.inv_dx), sy = (fabs(v) + c) * real(P.inv_dy);
  s = ok ? double(sx > sy ? sx : sy) : 0.0;
  return ok;
}

// Workgroup max of a non-negative double and OR of a flag, then one atomic each.
__device__ __forceinline__ void block_reduce_commit(double s, int bad, Ctrl* ctrl, int slot, int step_done) {
  __shared__ double red[16];
  __shared__ int redb[16];
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
    if (s > 0.0) atomicMax(&ctrl->smax_bits[slot], (unsigned long long)__double_as_longlong(s));
    if (bad) {
      if (atomicCAS(&ctrl->status, 0, 1) == 0) ctrl->fail_step = step_done;
    }
  }
}

template <class real>
__global__ __launch_bounds__(256) void k_update2(real* __restrict__ W, real* __restrict__ alpha,
                                                 const real* __restrict__ R, const real* __restrict__ FX,
                                                 const real* __restrict__ FY, Ctrl* __restrict__ ctrl, KParams P,
                                                 int step) {
  if (ctrl->status) return;
  const size_t N = (size_t)P.nx * P.ny, o = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  double s = 0.0;
  int bad = 0;
  if (o < N) {
    const int i = (int)(o % P.nx), j = (int)(o / P.nx);
    const real dt = real(ctrl->dt);
    real Lt[4], w[4];
    face_sum(FX, FY, P, i, j, 4, Lt);
    const real r3 = dt * dt * real(1.0 / 3.0);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      w[c] = R[c * N + o] + r3 * Lt[c];
      W[c * N + o] = w[c];
    }
    const int nx = P.nx, ny = P.ny;
    const size_t sx = (size_t)ny * (nx + 1), sy = (size_t)(ny + 1) * nx;
    const size_t fw = (size_t)j * (nx + 1) + i;
    const real* ax = FX + 8 * sx;
    const real* ay = FY + 8 * sy;
    alpha[o] = (ax[fw] * ax[fw + 1]) * (ay[o] * ay[o + nx]);
    bad = cell_speed(w, P, s) ? 0 : 1;
  }
  block_reduce_commit(s, bad, ctrl, (step + 1) & 1, step + 1);
}

template <class real>
__global__ __launch_bounds__(256) void k_speed(const real* __restrict__ W, Ctrl* __restrict__ ctrl, KParams P,
                                               int slot) {
  const size_t N = (size_t)P.nx * P.ny, o = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  double s = 0.0;
  int bad = 0;
  if (o < N) {
    real w[4] = {W[o], W[N + o], W[2 * N + o], W[3 * N + o]};
    bad = cell_speed(w, P, s) ? 0 : 1;
  }
  block_reduce_commit(s, bad, ctrl, slot, 0);
}

__global__ void k_ctrl_init(Ctrl* ctrl) {
  ctrl->smax_bits[0] = 0ull;
  ctrl->smax_bits[1] = 0ull;
  ctrl->dt = 0.0;
  ctrl->t = 0.0;
  ctrl->status = 0;
  ctrl->fail_step = -1;
}

template <class real>
__global__ __launch_bounds__(256) void k_assemble(const real* __restrict__ FX, const real* __restrict__ FY,
                                                  real* __restrict__ L, real* __restrict__ Lt,
                                                  real* __restrict__ an, KParams P) {
  const size_t N = (size_t)P.nx * P.ny, o = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= N) return;
  const int i = (int)(o % P.nx), j = (int)(o / P.nx);
  real a[4], b[4];
  face_sum(FX, FY, P, i, j, 0, a);
  face_sum(FX, FY, P, i, j, 4, b);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    L[c * N + o] = a[c];
    Lt[c * N + o] = b[c];
  }
  if (an) {
    const int nx = P.nx, ny = P.ny;
    const size_t sx = (size_t)ny * (nx + 1), sy = (size_t)(ny + 1) * nx;
    const size_t fw = (size_t)j * (nx + 1) + i;
    an[o] = (FX[8 * sx + fw] * FX[8 * sx + fw + 1]) * (FY[8 * sy + o] * FY[8 * sy + o + nx]);
  }
}

// ------------------------------------------------------------------------------------------------
// Host side.
// ------------------------------------------------------------------------------------------------
constexpr int kTF = 16, kTR = 28;

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
  if (a) hipEventRecord(a, st);
  launch();
  if (b) hipEventRecord(b, st);
  if (a && b) g_prof.recs.push_back({kind, a, b});
}

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
  off = align256(off + 9 * (size_t)g->ny * (g->nx + 1) * es);
  L.fy_off = off;
  off = align256(off + 9 * (size_t)(g->ny + 1) * g->nx * es);
  L.ctrl_off = off;
  off = align256(off + sizeof(Ctrl));
  L.total = off;
  return L;
}

static dfw_status check_common(const dfw_grid* g, const dfw_params* p, int32_t dtype) {
  if (!g || !p) return fail(DFW_EINVAL, "null grid or params");
  if (g->nx < 1 || g->ny < 1) return fail(DFW_EINVAL, "nx and ny must be >= 1");
  if ((size_t)g->nx * g->ny > ((size_t)1 << 31)) return fail(DFW_EINVAL, "grid too large (nx*ny > 2^31)");
  if (!(g->dx > 0) || !(g->dy > 0)) return fail(DFW_EINVAL, "dx and dy must be > 0");
  if ((g->bc_x != DFW_BC_PERIODIC && g->bc_x != DFW_BC_TRANSMISSIVE) ||
      (g->bc_y != DFW_BC_PERIODIC && g->bc_y != DFW_BC_TRANSMISSIVE))
    return fail(DFW_EINVAL, "unknown boundary condition");
  if (!(p->gamma > 1.0)) return fail(DFW_EINVAL, "gamma must be > 1");
  if (p->flux != DFW_FLUX_LF && p->flux != DFW_FLUX_GKS) return fail(DFW_EINVAL, "unknown flux");
  if (!(p->d_h > 0 && p->d_h < 1) || !(p->d_l >= 0 && p->d_l <= 1)) return fail(DFW_EINVAL, "d_h in (0,1), d_l in [0,1]");
  if (!(p->eps_weno > 0)) return fail(DFW_EINVAL, "eps_weno must be > 0");
  if (!(p->c1 >= 0) || !(p->c2 >= 0)) return fail(DFW_EINVAL, "c1, c2 must be >= 0");
  if (p->reserved != 0) return fail(DFW_EINVAL, "reserved must be 0");
  if (dtype != DFW_F64 && dtype != DFW_F32) return fail(DFW_EDTYPE, "dtype must be DFW_F64 or DFW_F32");
  return DFW_OK;
}

static KParams make_kparams(const dfw_grid* g, const dfw_params* p) {
  KParams P;
  P.nx = g->nx;
  P.ny = g->ny;
  P.bc_x = g->bc_x;
  P.bc_y = g->bc_y;
  P.dx = g->dx;
  P.dy = g->dy;
  P.inv_dx = 1.0 / g->dx;
  P.inv_dy = 1.0 / g->dy;
  P.gamma = p->gamma;
  P.cfl = p->cfl;
  P.dt_fixed = p->dt_fixed;
  P.alpha_thres = p->alpha_thres;
  P.eps = p->eps_weno;
  P.c1 = p->c1;
  P.c2 = p->c2;
  P.K = (4.0 - 2.0 * p->gamma) / (p->gamma - 1.0);
  P.d[3] = p->d_h;
  P.d[0] = (1.0 - p->d_h) * (1.0 - p->d_l) / 2.0;
  P.d[1] = (1.0 - p->d_h) * p->d_l;
  P.d[2] = P.d[0];
  return P;
}

#define HIP_TRY(x)                                                                          \
  do {                                                                                      \
    hipError_t e_ = (x);                                                                    \
    if (e_ != hipSuccess) return fail(DFW_EHIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

template <class real, int FLUX, int OUT>
static void launch_faces(const real* W, const real* A, real* FX, real* FY, Ctrl* ctrl, const KParams& P,
                         double dt_host, int lead, int step, double* dt_hist, hipStream_t st) {
  using T = Tile<kTF, kTR>;
  int nbx = ((P.nx + 1 + kTF - 1) / kTF) * ((P.ny + kTR - 1) / kTR);
  int nby = ((P.ny + 1 + kTF - 1) / kTF) * ((P.nx + kTR - 1) / kTR);
  hipLaunchKernelGGL((k_faces<real, FLUX, OUT, kTF, kTR>), dim3(nbx + nby), dim3(T::NT), 0, st, W, A, FX, FY,
                     ctrl, P, dt_host, lead, step, dt_hist);
}

template <class real, int OUT>
static void launch_faces_flux(int flux, const real* W, const real* A, real* FX, real* FY, Ctrl* ctrl,
                              const KParams& P, double dt_host, int lead, int step, double* dt_hist,
                              hipStream_t st) {
  if (flux == DFW_FLUX_LF) launch_faces<real, DFW_FLUX_LF, OUT>(W, A, FX, FY, ctrl, P, dt_host, lead, step, dt_hist, st);
  else launch_faces<real, DFW_FLUX_GKS, OUT>(W, A, FX, FY, ctrl, P, dt_host, lead, step, dt_hist, st);
}

static dim3 cell_grid(const KParams& P) { return dim3((unsigned)(((size_t)P.nx * P.ny + 255) / 256)); }

template <class real>
static dfw_status run_impl(real* W, real* A, const dfw_grid* g, const dfw_params* p, int nsteps, char* ws,
                           double* dt_hist, double* t_out, int32_t* fail_step, hipStream_t st) {
  WsLayout L = layout(g, sizeof(real));
  real* Ws = (real*)(ws + L.ws_off);
  real* R = (real*)(ws + L.r_off);
  real* FX = (real*)(ws + L.fx_off);
  real* FY = (real*)(ws + L.fy_off);
  Ctrl* ctrl = (Ctrl*)(ws + L.ctrl_off);
  KParams P = make_kparams(g, p);
  const double dth = p->dt_fixed > 0 ? p->dt_fixed : 0.0;
  hipLaunchKernelGGL(k_ctrl_init, dim3(1), dim3(1), 0, st, ctrl);
  timed(DFW_K_SPEED, st, [&] { hipLaunchKernelGGL(k_speed<real>, cell_grid(P), dim3(256), 0, st, W, ctrl, P, 0); });
  for (int n = 0; n < nsteps; ++n) {
    timed(DFW_K_FACES1, st, [&] {
      launch_faces_flux<real, OUT_F | OUT_FT>(p->flux, W, A, FX, FY, ctrl, P, dth, 1, n, dt_hist, st);
    });
    timed(DFW_K_UPDATE1, st, [&] {
      hipLaunchKernelGGL(k_update1<real>, cell_grid(P), dim3(256), 0, st, W, FX, FY, Ws, R, ctrl, P);
    });
    timed(DFW_K_FACES2, st, [&] {
      launch_faces_flux<real, OUT_FT | OUT_DF>(p->flux, Ws, A, FX, FY, ctrl, P, dth, 0, n, nullptr, st);
    });
    timed(DFW_K_UPDATE2, st, [&] {
      hipLaunchKernelGGL(k_update2<real>, cell_grid(P), dim3(256), 0, st, W, A, R, FX, FY, ctrl, P, n);
    });
  }
  HIP_TRY(hipGetLastError());
  Ctrl h;
  HIP_TRY(hipMemcpyAsync(&h, ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (t_out) *t_out = h.t;
  if (fail_step) *fail_step = h.status ? h.fail_step : -1;
  if (h.status) return fail(DFW_ENONPHYS, "non-physical state after " + std::to_string(h.fail_step) + " steps");
  return DFW_OK;
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

dfw_status dfw_run(void* W, void* alpha, const dfw_grid* grid, const dfw_params* params, int32_t nsteps,
                   int32_t dtype, void* ws, size_t ws_bytes, double* dt_hist_dev, double* t_out,
                   int32_t* fail_step, void* stream) {
  dfw_status s = check_common(grid, params, dtype);
  if (s != DFW_OK) return s;
  if (!W || !alpha) return fail(DFW_EINVAL, "W and alpha must be non-null");
  if (nsteps < 0) return fail(DFW_EINVAL, "nsteps must be >= 0");
  if (!(params->dt_fixed > 0) && !(params->cfl > 0)) return fail(DFW_EINVAL, "need cfl > 0 or dt_fixed > 0");
  if ((s = check_ws(grid, dtype, ws, ws_bytes)) != DFW_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  if (dtype == DFW_F64)
    return run_impl<double>((double*)W, (double*)alpha, grid, params, nsteps, (char*)ws, dt_hist_dev, t_out,
                            fail_step, st);
  return run_impl<float>((float*)W, (float*)alpha, grid, params, nsteps, (char*)ws, dt_hist_dev, t_out,
                         fail_step, st);
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
  KParams P = make_kparams(grid, params);
  hipLaunchKernelGGL(k_ctrl_init, dim3(1), dim3(1), 0, st, ctrl);
  if (dtype == DFW_F64) hipLaunchKernelGGL(k_speed<double>, cell_grid(P), dim3(256), 0, st, (const double*)W, ctrl, P, 0);
  else hipLaunchKernelGGL(k_speed<float>, cell_grid(P), dim3(256), 0, st, (const float*)W, ctrl, P, 0);
  HIP_TRY(hipGetLastError());
  Ctrl h;
  HIP_TRY(hipMemcpyAsync(&h, ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  double v;
  std::memcpy(&v, &h.smax_bits[0], sizeof(double));
  if (smax) *smax = v;
  if (nonphys) *nonphys = h.status ? 1 : 0;
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
  KParams P = make_kparams(grid, params);
  hipLaunchKernelGGL(k_ctrl_init, dim3(1), dim3(1), 0, st, ctrl);
  if (dtype == DFW_F64) {
    double* FX = (double*)((char*)ws + Lw.fx_off);
    double* FY = (double*)((char*)ws + Lw.fy_off);
    launch_faces_flux<double, OUT_F | OUT_FT | OUT_DF>(params->flux, (const double*)W, (const double*)alpha, FX, FY,
                                                       ctrl, P, dt, 0, 0, nullptr, st);
    hipLaunchKernelGGL(k_assemble<double>, cell_grid(P), dim3(256), 0, st, FX, FY, (double*)L, (double*)Lt,
                       (double*)alpha_new, P);
  } else {
    float* FX = (float*)((char*)ws + Lw.fx_off);
    float* FY = (float*)((char*)ws + Lw.fy_off);
    launch_faces_flux<float, OUT_F | OUT_FT | OUT_DF>(params->flux, (const float*)W, (const float*)alpha, FX, FY,
                                                      ctrl, P, dt, 0, 0, nullptr, st);
    hipLaunchKernelGGL(k_assemble<float>, cell_grid(P), dim3(256), 0, st, FX, FY, (float*)L, (float*)Lt,
                       (float*)alpha_new, P);
  }
  HIP_TRY(hipGetLastError());
  return DFW_OK;
}

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

const char* dfw_last_error(void) { return g_err.c_str(); }

}  // extern "C"
