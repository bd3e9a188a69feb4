"""ORACLE — test infrastructure, not part of the product.

Python (ctypes) access to the plain FP64 CPU reference in ``dfo.cpp`` of the S2O4 step with the
hybrid DF / WENO-AO reconstruction (Zhang, Ji & Xu, arXiv:2402.10914).  Only ``tests/``,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may import this package.  It
shares no code with the HIP implementation in ``paper_2402_10914_amd``.

Arrays are numpy float64, C-contiguous: W is [4, ny, nx] (rho, rho*U, rho*V, rho*E), alpha is
[ny, nx].
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "dfo.cpp")
LIB = os.path.join(HERE, "libdfo.so")

BC_PERIODIC, BC_TRANSMISSIVE = 0, 1
FLUX_LF, FLUX_GKS = 0, 1
TIME_S2O4, TIME_SSPRK3 = 0, 1


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (no fast-math, no FMA contraction, OpenMP over rows)."""
    if force or not os.path.exists(LIB):
        cmd = ["g++", "-std=c++17", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
               "-fPIC", "-shared", SRC, "-o", LIB + ".tmp"]
        subprocess.run(cmd, check=True)
        os.replace(LIB + ".tmp", LIB)
    return LIB


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("dx", ctypes.c_double),
                ("dy", ctypes.c_double), ("bc_x", ctypes.c_int32), ("bc_y", ctypes.c_int32)]


class Params(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("cfl", ctypes.c_double), ("dt_fixed", ctypes.c_double),
                ("alpha_thres", ctypes.c_double), ("d_h", ctypes.c_double), ("d_l", ctypes.c_double),
                ("eps_weno", ctypes.c_double), ("c1", ctypes.c_double), ("c2", ctypes.c_double),
                ("flux", ctypes.c_int32), ("time_limiter", ctypes.c_int32), ("time_scheme", ctypes.c_int32),
                ("t_end", ctypes.c_double), ("switch_rule", ctypes.c_int32), ("componentwise", ctypes.c_int32),
                ("df_stage", ctypes.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=False)
        L = ctypes.CDLL(LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        L.dfo_max_speed.restype = ctypes.c_int
        L.dfo_run.restype = ctypes.c_int
        L.dfo_smoothness.restype = ctypes.c_double
        L.dfo_limiter_weight.restype = ctypes.c_double
        L.dfo_df_gp.restype = ctypes.c_double
        L.dfo_moment.restype = ctypes.c_double
        L.dfo_moment.argtypes = [dp, ctypes.c_double, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                 ctypes.c_int32]
        L.dfo_df_gp.argtypes = [dp, dp, ctypes.c_double]
        L.dfo_smoothness.argtypes = [dp, ctypes.c_int32]
        L.dfo_u_moments.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int32, ctypes.c_int32, dp]
        L.dfo_char_basis.argtypes = [ctypes.c_int32, dp, ctypes.c_double, dp, dp]
        L.dfo_micro_slope.argtypes = [dp, dp, ctypes.c_double, dp]
        L.dfo_flux_gp.argtypes = [ctypes.c_int32, dp, dp, dp, dp, dp, dp, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_double, ctypes.c_double, dp, dp]
        L.dfo_rhs.argtypes = [dp, dp, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, dp, dp,
                              ctypes.c_void_p]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def make_grid(nx, ny, dx, dy, bc_x=BC_PERIODIC, bc_y=None) -> Grid:
    return Grid(int(nx), int(ny), float(dx), float(dy), int(bc_x), int(bc_x if bc_y is None else bc_y))


def make_params(flux=FLUX_LF, gamma=1.4, cfl=0.5, dt_fixed=0.0, alpha_thres=0.5, d_h=0.85, d_l=0.85,
                eps_weno=1e-6, c1=0.01, c2=5.0, time_limiter=0, time_scheme=TIME_S2O4, t_end=0.0,
                switch_rule=0, componentwise=0, df_stage=0) -> Params:
    return Params(float(gamma), float(cfl), float(dt_fixed), float(alpha_thres), float(d_h), float(d_l),
                  float(eps_weno), float(c1), float(c2), int(flux), int(time_limiter), int(time_scheme),
                  float(t_end), int(switch_rule), int(componentwise), int(df_stage))


def max_speed(W: np.ndarray, grid: Grid, params: Params):
    s = ctypes.c_double(0.0)
    rc = lib().dfo_max_speed(_p(W), ctypes.byref(grid), ctypes.byref(params), ctypes.byref(s))
    return s.value, rc == 0


def rhs(W, alpha, grid: Grid, params: Params, dt: float, want_alpha: bool = False):
    """Spatial operator of one stage: (L, dL/dt[, DF product from this stage's Gauss points])."""
    W = np.ascontiguousarray(W, dtype=np.float64)
    alpha = np.ascontiguousarray(alpha, dtype=np.float64)
    L = np.zeros_like(W)
    Lt = np.zeros_like(W)
    an = np.zeros_like(alpha) if want_alpha else None
    lib().dfo_rhs(_p(W), _p(alpha), ctypes.byref(grid), ctypes.byref(params), float(dt), _p(L), _p(Lt),
                  an.ctypes.data if an is not None else None)
    return (L, Lt, an) if want_alpha else (L, Lt)


def run(W, alpha, grid: Grid, params: Params, nsteps: int):
    """nsteps time steps (S2O4, or SSP-RK3 with params.time_scheme = TIME_SSPRK3), stopping at
    params.t_end when it is > 0.  Returns (W, alpha, t, dt_hist, fail_step) on copies of the inputs."""
    W = np.array(W, dtype=np.float64, order="C", copy=True)
    alpha = np.array(alpha, dtype=np.float64, order="C", copy=True)
    dt_hist = np.zeros(max(nsteps, 1))
    t = ctypes.c_double(0.0)
    fs = ctypes.c_int32(-1)
    lib().dfo_run(_p(W), _p(alpha), ctypes.byref(grid), ctypes.byref(params), int(nsteps), _p(dt_hist),
                  ctypes.byref(t), ctypes.byref(fs))
    return W, alpha, t.value, dt_hist[:nsteps], fs.value


def run_tangent(W, alpha, dW, dalpha, grid: Grid, params: Params, dt_hist):
    """Forward-mode directional derivative of len(dt_hist) steps with frozen time steps."""
    W = np.array(W, dtype=np.float64, order="C", copy=True)
    alpha = np.array(alpha, dtype=np.float64, order="C", copy=True)
    dW = np.array(dW, dtype=np.float64, order="C", copy=True)
    dalpha = np.array(dalpha, dtype=np.float64, order="C", copy=True)
    dt_hist = np.ascontiguousarray(dt_hist, dtype=np.float64)
    lib().dfo_run_tangent(_p(W), _p(alpha), _p(dW), _p(dalpha), ctypes.byref(grid), ctypes.byref(params),
                          int(len(dt_hist)), _p(dt_hist))
    return W, alpha, dW, dalpha


# ---- unit-level access (pins) ----

def candidate(k: int) -> np.ndarray:
    c = np.zeros(25)
    lib().dfo_candidate(int(k), _p(c))
    return c.reshape(5, 5)


def smoothness(coef, deg: int) -> float:
    c = np.zeros(5)
    c[: len(coef)] = coef
    return lib().dfo_smoothness(_p(c), int(deg))


def weno_ao(Q, params: Params) -> np.ndarray:
    Q = np.ascontiguousarray(Q, dtype=np.float64)
    P = np.zeros(5)
    lib().dfo_weno_ao(_p(Q), ctypes.byref(params), _p(P))
    return P


def limiter_weight(Q, params: Params) -> float:
    """Non-linear time-limiter weight of eq. (29) for one five-average stencil."""
    Q = np.ascontiguousarray(Q, dtype=np.float64)
    return lib().dfo_limiter_weight(_p(Q), ctypes.byref(params))


def hybrid(Q, a3, params: Params) -> np.ndarray:
    Q = np.ascontiguousarray(Q, dtype=np.float64)
    a3 = np.ascontiguousarray(a3, dtype=np.float64)
    P = np.zeros(5)
    lib().dfo_hybrid(_p(Q), _p(a3), ctypes.byref(params), _p(P))
    return P


def char_basis(direction: int, W, gamma=1.4):
    W = np.ascontiguousarray(W, dtype=np.float64)
    R = np.zeros(16)
    L = np.zeros(16)
    lib().dfo_char_basis(int(direction), _p(W), float(gamma), _p(R), _p(L))
    return R.reshape(4, 4), L.reshape(4, 4)


def flux_gp(flux, Wl, Wlx, Wly, Wr, Wrx, Wry, gamma=1.4, dt=1e-3, c1=0.01, c2=5.0):
    a = [np.ascontiguousarray(x, dtype=np.float64) for x in (Wl, Wlx, Wly, Wr, Wrx, Wry)]
    F = np.zeros(4)
    Ft = np.zeros(4)
    lib().dfo_flux_gp(int(flux), *[_p(x) for x in a], float(gamma), float(dt), float(c1), float(c2),
                      _p(F), _p(Ft))
    return F, Ft


def df_gp(Wl, Wr, gamma=1.4) -> float:
    return lib().dfo_df_gp(_p(np.ascontiguousarray(Wl, dtype=np.float64)),
                           _p(np.ascontiguousarray(Wr, dtype=np.float64)), float(gamma))


def u_moments(U, lam, space, n=8) -> np.ndarray:
    M = np.zeros(n)
    lib().dfo_u_moments(float(U), float(lam), int(space), int(n), _p(M))
    return M


def micro_slope(W, dW, gamma=1.4) -> np.ndarray:
    a = np.zeros(4)
    lib().dfo_micro_slope(_p(np.ascontiguousarray(W, dtype=np.float64)),
                          _p(np.ascontiguousarray(dW, dtype=np.float64)), float(gamma), _p(a))
    return a


def moment(W, space, a, b, c, gamma=1.4) -> float:
    return lib().dfo_moment(_p(np.ascontiguousarray(W, dtype=np.float64)), float(gamma), int(space),
                            int(a), int(b), int(c))
