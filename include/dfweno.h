/*
 * dfweno.h — C ABI of the MI355X (gfx950) implementation of one two-stage fourth-order (S2O4)
 * time step of the 2-D Euler finite-volume scheme with the hybrid discontinuity-feedback (DF) /
 * WENO-AO reconstruction of Zhang, Ji & Xu, "A robustness-enhanced reconstruction based on
 * discontinuity feedback factor for high-order finite volume scheme" (arXiv:2402.10914).
 *
 * Problem statement (Algorithm 1 of the paper): input the cell averages W^n and the DF field
 * alpha^n, output W^{n+1} and alpha^{n+1}; the time increment comes from the CFL condition.
 *
 * Conventions shared by every entry point
 *   - Array pointers marked "device" point to device memory owned by the caller; the library
 *     never allocates, frees or retains them beyond the call.  Host pointers are marked "host".
 *   - W is [4][ny][nx] contiguous, component-major: rho, rho*U, rho*V, rho*E (cell averages).
 *     alpha is [ny][nx] contiguous.  Both have the element type given by `dtype` (DFW_F64 or
 *     DFW_F32); cell (i, j) is at offset j*nx + i.
 *   - `stream` is a hipStream_t passed as void*; NULL means the default stream.  Work is
 *     enqueued in stream order; calls that return host values synchronise that stream once.
 *   - `ws` is a device workspace of at least dfw_workspace_bytes() bytes, 256-byte aligned.
 *   - Every call returns a dfw_status; on a non-OK status dfw_last_error() returns a message
 *     (thread-local, valid until the next call on the same thread).
 */
#ifndef DFWENO_H
#define DFWENO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DFW_OK = 0,
  DFW_EINVAL = 1,      /* invalid argument (null pointer, size, unknown flux/bc/dtype, gamma <= 1, ...) */
  DFW_EDTYPE = 2,      /* unsupported element type */
  DFW_EWORKSPACE = 3,  /* workspace missing, misaligned or too small */
  DFW_EHIP = 4,        /* a HIP runtime call failed */
  DFW_ENONPHYS = 5     /* a state with rho <= 0, p <= 0 or a non-finite value was met */
} dfw_status;

enum { DFW_FLUX_LF = 0, DFW_FLUX_GKS = 1 };        /* Section 2.3 (Lax-Friedrichs), Section 2.2 (gas-kinetic) */
enum { DFW_BC_PERIODIC = 0, DFW_BC_TRANSMISSIVE = 1 };
enum { DFW_F64 = 0, DFW_F32 = 1 };
enum { DFW_TIME_S2O4 = 0, DFW_TIME_SSPRK3 = 1 };  /* eq. (21) (Section 2.2), eq. (32) (Section 2.3) */

/* Uniform structured grid: nx by ny cells of size dx by dy; one boundary type per axis.
 * Transmissive = ghost cells copy the nearest interior cell (the free boundary of Section 4). */
typedef struct {
  int32_t nx, ny;
  double dx, dy;
  int32_t bc_x, bc_y;
} dfw_grid;

/* Scheme parameters (defaults of the paper in brackets).
 *   gamma        ratio of specific heats [1.4]
 *   cfl          dt = cfl / max over cells of max((|U|+c)/dx, (|V|+c)/dy)   [0.5]
 *   dt_fixed     if > 0, every step uses this dt instead of the CFL condition
 *   alpha_thres  DF threshold of the hybrid switch, eq. (42), strict "<" [0.5]
 *   d_h, d_l     linear-weight parameters of WENO-AO (Section 3.1) [0.85, 0.85]
 *   eps_weno     epsilon of the WENO-Z weights (not given by the paper) [1e-6]
 *   c1, c2       numerical collision time tau_n = c1 dt + c2 |(pl-pr)/(pl+pr)| dt (Section 2.2) [0.01, 5]
 *   flux         DFW_FLUX_LF or DFW_FLUX_GKS
 *   tile         interface tile shape, 0 <= tile < dfw_num_tiles() [0]; results do not depend on it
 *   time_limiter 1: the non-linear time limiter of Section 2.2 (eqs. (27)-(29)) for the second-stage
 *                update; 0: plain eq. (21) [0].  The limiter's epsilon is eps_weno.  dfw_rhs
 *                returns the unlimited dL/dt; dfw_adjoint rejects time_limiter = 1.
 *   time_scheme  DFW_TIME_S2O4: the two-stage fourth-order step of eq. (21) [default];
 *                DFW_TIME_SSPRK3: the three-stage SSP Runge-Kutta step of eq. (32), which needs no
 *                flux time derivative.  As in the paper it runs with the LF flux only (GKS, or
 *                the time limiter, with it are rejected with DFW_EINVAL).  dt comes from the CFL
 *                condition on W^n, alpha^n drives the hybrid switch in all three stages and
 *                alpha^{n+1} is built from the third stage's Gauss points.  dfw_adjoint covers
 *                DFW_TIME_S2O4 only.
 *   t_end        > 0: the run stops at time t_end.  The step that would pass it is shortened to
 *                end exactly on t_end (so the returned t equals t_end) and any remaining steps
 *                are skipped and record dt = 0 in dt_hist; nsteps is then an upper bound on the
 *                steps taken.  0: exactly nsteps steps [0].  Must be >= 0; dfw_adjoint requires 0.
 *   switch_rule  0: the hybrid switch of eq. (42) as printed, DF quadratic when the largest DF
 *                value of the cell and its two neighbours is below alpha_thres [0]; 1: when the
 *                smallest is (a discontinuity in any of the three cells); 2: when the cell's own
 *                value is.  Options for ablations and the robustness sweeps; the adjoint follows
 *                the same rule.
 *   componentwise 0: reconstruct characteristic variables (eigenvectors of the normal flux
 *                Jacobian at the mean of the two cells beside each interface) [0]; 1: reconstruct
 *                the conservative variables component by component (ablation).
 *   df_stage     0: alpha^{n+1} from the Gauss-point states of the last stage [0]; 1: from the
 *                first stage's (the states of W^n; ablation).  dfw_adjoint requires both 0. */
typedef struct {
  double gamma, cfl, dt_fixed, alpha_thres, d_h, d_l, eps_weno, c1, c2;
  int32_t flux;
  int32_t tile;
  int32_t time_limiter;
  int32_t time_scheme;
  double t_end;
  int32_t switch_rule;
  int32_t componentwise;
  int32_t df_stage;
} dfw_params;

/* Bytes of device workspace needed by dfw_run / dfw_rhs / dfw_max_speed for this grid. */
size_t dfw_workspace_bytes(const dfw_grid* grid, int32_t dtype);

/* Advance (W, alpha) in place by nsteps time steps: S2O4 (eq. (21); Algorithm 1), or SSP-RK3
 * (eq. (32)) when params->time_scheme says so.
 *   W, alpha        device, in/out.
 *   dt_hist_dev     device, optional (may be NULL): receives the nsteps time increments (FP64).
 *   t_out           host, optional: the time reached (sum of the increments taken; t_end exactly
 *                   when the run reached it).
 *   fail_step       host, optional: -1 on success; otherwise the number of completed steps when
 *                   a non-physical state was found (0 = the input).  W then holds that state and
 *                   later steps are skipped; the call returns DFW_ENONPHYS.
 * Synchronises `stream` once at the end. */
dfw_status dfw_run(void* W, void* alpha, const dfw_grid* grid, const dfw_params* params, int32_t nsteps,
                   int32_t dtype, void* ws, size_t ws_bytes, double* dt_hist_dev, double* t_out,
                   int32_t* fail_step, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): dfw_run with its workspace in a fixed device array of
 * DFW_NOALLOC_SCRATCH_BYTES bytes inside the library instead of a caller-provided one.  Same
 * arguments, results and synchronisation as dfw_run, minus ws / ws_bytes.  Calls no hipMalloc,
 * hipFree or other allocating routine.
 *   Limit: dfw_workspace_bytes(grid, dtype) must not exceed DFW_NOALLOC_SCRATCH_BYTES (64 MiB: up to
 *   about 299 000 cells in FP64, e.g. 512 x 512; about 599 000 in FP32); larger grids return
 *   DFW_EWORKSPACE before anything is launched.
 *   The array is per GPU (the current device; `stream` must belong to it), allocated when the
 *   library is loaded and held until the process ends; its address is looked up once per device at
 *   the first call there.  Every call on a GPU shares that GPU's array and leaves its contents
 *   behind; each call initialises the part that must start at zero (the control block) with a
 *   kernel of its own.  Calls that overlap on one GPU (other streams or threads) race on the array
 *   and must be serialised by the caller. */
#define DFW_NOALLOC_SCRATCH_BYTES (64u << 20)
dfw_status dfw_run_noalloc(void* W, void* alpha, const dfw_grid* grid, const dfw_params* params, int32_t nsteps,
                           int32_t dtype, double* dt_hist_dev, double* t_out, int32_t* fail_step, void* stream);

/* The CFL reduction alone (Algorithm 1, the step that sets the time increment from the CFL
 * condition; the paper gives no formula, so dt = cfl / smax with
 * smax = max over cells of max((|U|+c)/dx, (|V|+c)/dy), c = sqrt(gamma p / rho)).
 *   W device in, [4][ny][nx]; smax (host, FP64) out; nonphys (host) out: 1 if any cell has
 *   rho <= 0, p <= 0 or a non-finite value (those cells do not enter smax), else 0.
 *   ws: the dfw_run workspace (its control block is used).  Synchronises `stream`. */
dfw_status dfw_max_speed(const void* W, const dfw_grid* grid, const dfw_params* params, int32_t dtype,
                         void* ws, size_t ws_bytes, double* smax, int32_t* nonphys, void* stream);

/* The spatial operator of one stage, eqs. (3)-(4) with its time derivative (Section 2.2): for the
 * state W and DF field alpha, writes L(W) and dL/dt(W) ([4][ny][nx], device) and, if alpha_new
 * is non-NULL, the DF product of every cell built from this stage's Gauss-point states
 * ([ny][nx], device).  dt is used only by the gas-kinetic flux.  Stream-ordered, no sync. */
dfw_status dfw_rhs(const void* W, const void* alpha, const dfw_grid* grid, const dfw_params* params,
                   int32_t dtype, double dt, void* L, void* Lt, void* alpha_new, void* ws, size_t ws_bytes,
                   void* stream);

/* ---- Batched ragged grids ---------------------------------------------------------------------
 * Many independent grids (own sizes, spacing, boundaries and CFL time steps; one dfw_params for
 * all) advanced together: every kernel launch covers the interfaces or cells of all grids, and
 * dfw_batch_run can capture the whole nsteps rollout once into a hipGraph and replay it with one
 * launch.  The states are packed back to back: grid g's W ([4][ny_g][nx_g]) starts at element
 * w_offsets[g] of W_flat and its alpha at a_offsets[g] of alpha_flat (dfw_batch_layout). */
typedef struct dfw_batch dfw_batch;

/* Sweep order of the interface tiles of a batch (an autotuning knob; results do not depend on it). */
enum { DFW_ORDER_GRID = 0, DFW_ORDER_LARGEST_FIRST = 1, DFW_ORDER_INTERLEAVED = 2 };

/* Builds the descriptor and tile tables (host and a small device copy owned by the plan). */
dfw_status dfw_batch_plan(const dfw_grid* grids, int32_t ngrids, const dfw_params* params, int32_t dtype,
                          int32_t order, dfw_batch** out);

/* Offsets (elements, host arrays of ngrids, may be NULL) and total sizes of the packed layout and
 * the workspace the plan needs. */
dfw_status dfw_batch_layout(const dfw_batch* b, int64_t* w_offsets, int64_t* a_offsets, size_t* w_elems,
                            size_t* a_elems, size_t* ws_bytes);

/* Advances every grid by nsteps S2O4 steps in place.  use_graph != 0 replays a hipGraph captured
 * at the first call with these pointers and nsteps (re-captured when they change).
 *   dt_hist_dev  device, optional: [ngrids][nsteps] FP64 time increments.
 *   t_out        host, optional: [ngrids] simulated time of each grid.
 *   fail_steps   host, optional: [ngrids] -1 or the completed steps when that grid met a
 *                non-physical state (the other grids continue); returns DFW_ENONPHYS if any. */
dfw_status dfw_batch_run(dfw_batch* b, void* W_flat, void* alpha_flat, int32_t nsteps, void* ws, size_t ws_bytes,
                         int32_t use_graph, double* dt_hist_dev, double* t_out, int32_t* fail_steps, void* stream);

void dfw_batch_free(dfw_batch* b);

/* ---- Reverse mode (adjoint) -------------------------------------------------------------------
 * The gradient of a scalar loss J(W^N, alpha^N) of an N-step rollout (eq. (21) steps, Section 3)
 * with respect to its initial state (W^0, alpha^0), by the hand-written adjoint of every operation
 * of the step: characteristic projection, WENO-AO(5,3) with WENO-Z weights and the DF hybrid
 * (Section 3.1, eqs. (33)-(39); Section 3.3, eqs. (42)-(43)), the DF factor (Section 3.2, eqs. (40)-(41)), the LF and GKS fluxes and
 * their time derivatives (Section 2), and the two S2O4 stages.  The time steps are held fixed at a
 * recorded dt history (the CFL reduction is not differentiated).  Kinks follow one fixed
 * subgradient convention: d|x|/dx = sign(x) with sign(0) = 0; max(a, b) follows a when a >= b; the
 * switch of eq. (42) contributes no derivative (the branch taken is differentiated).
 *
 * Memory: dfw_run_ckpt stores (W, alpha) at every ckpt_every-th step; dfw_adjoint recomputes one
 * segment of ckpt_every steps at a time from its checkpoint and reverses it.  ckpt_every = 1 stores
 * each step's whole record instead (W^n, alpha^n, the first-stage state W* and the second-stage
 * interface DF products: about 11 N values per step, N = nx ny), and dfw_adjoint recomputes
 * nothing; the gradient is bitwise the same for every ckpt_every.  The adjoint is FP64 (dtype
 * DFW_F64; DFW_F32 gives DFW_EDTYPE).  Deterministic: no atomics, results are bitwise
 * reproducible. */

/* Bytes of the checkpoint store of an nsteps rollout (0 for invalid arguments). */
size_t dfw_checkpoint_bytes(const dfw_grid* grid, int32_t dtype, int32_t nsteps, int32_t ckpt_every);

/* dfw_run (same arguments and results) that also writes checkpoints to ckpt (device, owned by the
 * caller, >= dfw_checkpoint_bytes, 256-byte aligned).  dt_hist_dev is required here: it records
 * the time steps the adjoint is taken at. */
dfw_status dfw_run_ckpt(void* W, void* alpha, const dfw_grid* grid, const dfw_params* params, int32_t nsteps,
                        int32_t dtype, int32_t ckpt_every, void* ckpt, size_t ckpt_bytes, void* ws,
                        size_t ws_bytes, double* dt_hist_dev, double* t_out, int32_t* fail_step, void* stream);

/* Workspace bytes of dfw_adjoint (0 for invalid arguments); about (11 ckpt_every + 70) N values,
 * 70 N for ckpt_every = 1. */
size_t dfw_adjoint_workspace_bytes(const dfw_grid* grid, int32_t dtype, int32_t ckpt_every);

/* Adjoint of the rollout recorded by dfw_run_ckpt (same grid, params, nsteps, ckpt_every; ckpt and
 * dt_hist_dev as it wrote them).  In: gW_final = dJ/dW^N ([4][ny][nx]), gA_final = dJ/dalpha^N
 * ([ny][nx]; NULL means zero).  Out: gW0 = dJ/dW^0, gA0 = dJ/dalpha^0 (NULL: not written).  All
 * device pointers; the outputs may not alias the inputs or the workspace.  Stream-ordered; waits
 * for the stream once at the end.  DFW_ENONPHYS if the recomputed forward meets a non-physical
 * state (a dt_hist other than the recorded one). */
dfw_status dfw_adjoint(const dfw_grid* grid, const dfw_params* params, int32_t dtype, int32_t nsteps,
                       int32_t ckpt_every, const void* ckpt, size_t ckpt_bytes, const double* dt_hist_dev,
                       const void* gW_final, const void* gA_final, void* gW0, void* gA0, void* ws, size_t ws_bytes,
                       void* stream);

/* Interface tile shapes available for dfw_params.tile: TF interfaces by TR segments. */
int32_t dfw_num_tiles(void);
dfw_status dfw_tile_shape(int32_t tile, int32_t* tf, int32_t* tr);

/* Measurement support: per-kernel device time of the launches made by dfw_run, recorded with HIP
 * events on the stream the kernels run on.  Kernel kinds index the arrays of dfw_profile_read. */
enum {
  DFW_K_FACES1 = 0,   /* interface kernel, first stage (flux and time derivative) */
  DFW_K_UPDATE1 = 1,  /* cell kernel, first stage (W*, and the S2O4 accumulator) */
  DFW_K_FACES2 = 2,   /* interface kernel, second stage (time derivative and DF) */
  DFW_K_UPDATE2 = 3,  /* cell kernel, second stage (W^{n+1}, alpha^{n+1}, CFL reduction) */
  DFW_K_SPEED = 4,    /* standalone CFL reduction of the input state */
  DFW_K_GRAPH = 5,    /* one replay of a captured batched rollout */
  DFW_K_ADJ_FACES1 = 6, /* adjoint interface kernel, first stage */
  DFW_K_ADJ_FACES2 = 7, /* adjoint interface kernel, second stage */
  DFW_K_ADJ_GATHER = 8, /* adjoint cell gather (both stages) */
  DFW_K_RK_FACES = 9,   /* interface kernel of an SSP-RK3 stage (flux; DF in the third stage) */
  DFW_K_RK_UPDATE = 10, /* cell kernel of an SSP-RK3 stage (the third with alpha^{n+1} and CFL reduction) */
  DFW_K_COUNT = 11
};

/* enable != 0 clears the records and starts recording; 0 stops.  Process-wide, not thread-safe;
 * meant for benchmarks only (recording adds two events per launch). */
dfw_status dfw_profile(int32_t enable);

/* Synchronises the recorded events and writes, for each kind k < n, the summed device time in
 * milliseconds (ms[k], host) and the number of launches (launches[k], host). */
dfw_status dfw_profile_read(double* ms, int64_t* launches, int32_t n);

/* Message for the last non-OK status returned on this thread. */
const char* dfw_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DFWENO_H */
