"""Seeded synthetic inputs for the S2O4 DF-hybrid step (shared by the tests, the smoke check and
the benchmark).

This module holds initial conditions only — none of the scheme's arithmetic.  Every array is built
on the host with numpy from an explicit seed (``numpy.random.default_rng``, PCG64), so the HIP path
and the CPU oracle always receive identical bytes.

Layout: W is float64 [4, ny, nx] holding cell averages of (rho, rho*U, rho*V, rho*E); the DF field
alpha is float64 [ny, nx] and starts at 1 (the first step is pure WENO-AO).

Workloads (the paper's test problems are analytic, so no dataset is involved):
  * ``density_wave``   advected wave rho = 1 + 0.2 sin(pi (x + y)), U = V = 1, p = 1 on [0,2]^2,
                       exact cell averages; the exact solution is the same wave shifted by (t, t).
  * ``product_wave``   the paper's 2-D accuracy problem rho = 1 + 0.2 sin(pi x) sin(pi y) on
                       [-1,1]^2 (Section 4.1), exact cell averages.
  * ``sine_wave_1d``   the paper's 1-D accuracy problem rho = 1 + 0.2 sin(pi x) on [0,2] (ny = 1).
  * ``riemann4``       four-quadrant piecewise-constant data split at a random point in
                       [0.3,0.7]^2, per quadrant rho~U[0.1,2], U,V~U[-1,1], p~U[0.05,1.5]
                       (stand-in for the paper's 2-D Riemann configurations).
  * ``circles``        density-wave background plus seeded circular regions with density ratios up
                       to 10 and pressure ratios up to 1e3.
  * ``batch``          ragged set of independent grids (half density wave, half Riemann).
  * ``bumps``          density wave plus seeded Gaussian bumps (adjoint workload) and its target.
  * ``problem_123``, ``hurricane``, ``rarefaction2d``
                       the robustness problems of Section 4.3, each parameterised by its reference
                       Mach number (Tables 5-7 report the largest Mach number a scheme survives).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

GAMMA = 1.4
BC_PERIODIC, BC_TRANSMISSIVE = 0, 1
FLUX_LF, FLUX_GKS = 0, 1


@dataclass
class Problem:
    """A grid plus its initial state and the run settings of one workload."""
    name: str
    nx: int
    ny: int
    x0: float
    y0: float
    dx: float
    dy: float
    bc_x: int
    bc_y: int
    W: np.ndarray
    alpha: np.ndarray
    flux: int = FLUX_LF
    cfl: float = 0.5
    nsteps: int = 1
    gamma: float = GAMMA
    extra: dict = field(default_factory=dict)


def _sinc_avg(h: float) -> float:
    """Cell average of sin(pi (x_c + s)) over a cell of width h equals sin(pi x_c) * S(h)."""
    a = math.pi * h / 2.0
    return math.sin(a) / a


def _centres(n: int, x0: float, d: float) -> np.ndarray:
    return x0 + (np.arange(n) + 0.5) * d


def _assemble(rho, u, v, p, gamma=GAMMA) -> np.ndarray:
    """Conservative point values (or cell averages when U, V, p are constant)."""
    W = np.empty((4,) + rho.shape, dtype=np.float64)
    W[0] = rho
    W[1] = rho * u
    W[2] = rho * v
    W[3] = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)
    return W


def density_wave_avg(nx, ny, t=0.0, x0=0.0, y0=0.0, lx=2.0, ly=2.0):
    """Exact cell averages of rho = 1 + 0.2 sin(pi (x + y - 2 t))."""
    dx, dy = lx / nx, ly / ny
    xc = _centres(nx, x0, dx)
    yc = _centres(ny, y0, dy)
    ph = np.pi * (xc[None, :] + yc[:, None] - 2.0 * t)
    return 1.0 + 0.2 * np.sin(ph) * _sinc_avg(dx) * _sinc_avg(dy)


def density_wave(nx=64, ny=None, gamma=GAMMA, flux=FLUX_LF, cfl=0.5, nsteps=20) -> Problem:
    ny = nx if ny is None else ny
    rho = density_wave_avg(nx, ny)
    one = np.ones_like(rho)
    W = _assemble(rho, one, one, one, gamma)  # U, V, p constant: averages are exact
    return Problem("density_wave", nx, ny, 0.0, 0.0, 2.0 / nx, 2.0 / ny, BC_PERIODIC, BC_PERIODIC, W,
                   np.ones((ny, nx)), flux=flux, cfl=cfl, nsteps=nsteps, gamma=gamma)


def product_wave_avg(n, t=0.0):
    """Exact cell averages of rho = 1 + 0.2 sin(pi (x - t)) sin(pi (y - t)) on [-1,1]^2."""
    d = 2.0 / n
    c = _centres(n, -1.0, d)
    sx = np.sin(np.pi * (c - t)) * _sinc_avg(d)
    return 1.0 + 0.2 * sx[None, :] * sx[:, None]


def product_wave(n, gamma=GAMMA, flux=FLUX_GKS) -> Problem:
    rho = product_wave_avg(n)
    one = np.ones_like(rho)
    W = _assemble(rho, one, one, one, gamma)
    return Problem("product_wave", n, n, -1.0, -1.0, 2.0 / n, 2.0 / n, BC_PERIODIC, BC_PERIODIC, W,
                   np.ones((n, n)), flux=flux, gamma=gamma)


def sine_wave_1d_avg(n, t=0.0):
    d = 2.0 / n
    c = _centres(n, 0.0, d)
    return 1.0 + 0.2 * np.sin(np.pi * (c - t)) * _sinc_avg(d)


def sine_wave_1d(n, gamma=GAMMA, flux=FLUX_GKS) -> Problem:
    """ny = 1 periodic strip (dy = dx) carrying the 1-D sine wave with U = 1, V = 0, p = 1."""
    rho = sine_wave_1d_avg(n)[None, :]
    one = np.ones_like(rho)
    W = _assemble(rho, one, 0.0 * one, one, gamma)
    d = 2.0 / n
    return Problem("sine_wave_1d", n, 1, 0.0, 0.0, d, d, BC_PERIODIC, BC_PERIODIC, W, np.ones((1, n)),
                   flux=flux, gamma=gamma)


def _riemann_states(rng, gamma):
    """Draw four quadrant states (SW, SE, NE, NW); redraw if an edge 1-D Riemann problem would
    create vacuum (u_R - u_L >= 2 (c_L + c_R) / (gamma - 1))."""
    while True:
        rho = rng.uniform(0.1, 2.0, 4)
        u = rng.uniform(-1.0, 1.0, 4)
        v = rng.uniform(-1.0, 1.0, 4)
        p = rng.uniform(0.05, 1.5, 4)
        c = np.sqrt(gamma * p / rho)
        SW, SE, NE, NW = 0, 1, 2, 3
        pairs = [(SW, SE, u), (NW, NE, u), (SW, NW, v), (SE, NE, v)]
        ok = all(vel[b] - vel[a] < 2.0 * (c[a] + c[b]) / (gamma - 1.0) for a, b, vel in pairs)
        if ok:
            return rho, u, v, p


def riemann4(n=512, ny=None, seed=2402, gamma=GAMMA, flux=FLUX_GKS, cfl=0.4, nsteps=200) -> Problem:
    ny = n if ny is None else ny
    rng = np.random.default_rng(seed)
    xs, ys = rng.uniform(0.3, 0.7, 2)
    rho_q, u_q, v_q, p_q = _riemann_states(rng, gamma)
    dx, dy = 1.0 / n, 1.0 / ny
    xc = _centres(n, 0.0, dx)[None, :]
    yc = _centres(ny, 0.0, dy)[:, None]
    east = xc >= xs
    north = yc >= ys
    q = np.where(~north & ~east, 0, np.where(~north & east, 1, np.where(north & east, 2, 3)))
    W = _assemble(rho_q[q], u_q[q], v_q[q], p_q[q], gamma)
    return Problem("riemann4", n, ny, 0.0, 0.0, dx, dy, BC_TRANSMISSIVE, BC_TRANSMISSIVE, W,
                   np.ones((ny, n)), flux=flux, cfl=cfl, nsteps=nsteps, gamma=gamma,
                   extra={"split": (xs, ys), "seed": seed})


def circles(n=4096, seed=10914, ncirc=32, edge_cells=2.0, gamma=GAMMA, flux=FLUX_LF, cfl=0.4,
            nsteps=50) -> Problem:
    """Point-sampled density-wave background (U = V = 1, p = 1) on periodic [0,2]^2 with ncirc
    circular regions: centre ~U[0,2]^2, radius R ~U[0.01,0.05], density factor 10^U[-1,1] over the
    background and pressure 10^U[0,3].  Each region has a smooth edge
    f(r) = (1 - tanh((r - R) / w)) / 2 with w = edge_cells * dx (periodic minimum-image distance),
    and later regions overwrite earlier ones by geometric blending:
        log q <- (1 - f) log q + f log q_region   (q = rho, p).
    The smooth edge keeps the initial WENO reconstruction from producing negative Gauss-point
    pressures at the sharpest (pressure ratio 1e3) edges, which the scheme has no limiter for.
    edge_cells = 0 gives the sharp, point-sampled regions (f = 1 where r <= R, else 0)."""
    rng = np.random.default_rng(seed)
    d = 2.0 / n
    xc = _centres(n, 0.0, d)[None, :]
    yc = _centres(n, 0.0, d)[:, None]
    rho_bg = 1.0 + 0.2 * np.sin(np.pi * (xc + yc))
    lrho = np.log(rho_bg)
    lp = np.zeros((n, n))
    w = edge_cells * d
    for _ in range(ncirc):
        cx, cy = rng.uniform(0.0, 2.0, 2)
        r = rng.uniform(0.01, 0.05)
        rfac = 10.0 ** rng.uniform(-1.0, 1.0)
        pin = 10.0 ** rng.uniform(0.0, 3.0)
        ddx = np.abs(xc - cx)
        ddx = np.minimum(ddx, 2.0 - ddx)
        ddy = np.abs(yc - cy)
        ddy = np.minimum(ddy, 2.0 - ddy)
        dist = np.sqrt(ddx * ddx + ddy * ddy)
        f = (dist <= r).astype(np.float64) if edge_cells <= 0 else 0.5 * (1.0 - np.tanh((dist - r) / w))
        lrho = (1.0 - f) * lrho + f * np.log(rho_bg * rfac)
        lp = (1.0 - f) * lp + f * np.log(pin)
    rho = np.exp(lrho)
    p = np.exp(lp)
    one = np.ones((n, n))
    W = _assemble(rho, one, one, p, gamma)
    return Problem("circles", n, n, 0.0, 0.0, d, d, BC_PERIODIC, BC_PERIODIC, W, np.ones((n, n)),
                   flux=flux, cfl=cfl, nsteps=nsteps, gamma=gamma, extra={"seed": seed})


def batch(ngrids=256, seed=256, lo=32, hi=512, gamma=GAMMA, flux=FLUX_LF, cfl=0.4, nsteps=100):
    """Ragged batch: side lengths round(exp(U[ln lo, ln hi])) drawn independently for nx and ny;
    even grids carry the density wave (periodic [0,2]^2), odd grids four-quadrant Riemann data
    (transmissive [0,1]^2, seed (seed, g))."""
    rng = np.random.default_rng(seed)
    sizes = np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), (ngrids, 2)))).astype(int)
    probs = []
    for g in range(ngrids):
        nx, ny = int(sizes[g, 0]), int(sizes[g, 1])
        if g % 2 == 0:
            pr = density_wave(nx, ny, gamma=gamma, flux=flux, cfl=cfl, nsteps=nsteps)
        else:
            pr = riemann4(nx, ny, seed=[seed, g], gamma=gamma, flux=flux, cfl=cfl, nsteps=nsteps)
        probs.append(pr)
    return probs


def _bump_field(n, rng, nbumps, amp, width):
    d = 2.0 / n
    xc = _centres(n, 0.0, d)[None, :]
    yc = _centres(n, 0.0, d)[:, None]
    f = np.zeros((n, n))
    for _ in range(nbumps):
        cx, cy = rng.uniform(0.0, 2.0, 2)
        ddx = np.abs(xc - cx)
        ddx = np.minimum(ddx, 2.0 - ddx)
        ddy = np.abs(yc - cy)
        ddy = np.minimum(ddy, 2.0 - ddy)
        f += amp * np.exp(-(ddx * ddx + ddy * ddy) / (2.0 * width * width))
    return f


def bumps(n=1024, seed=1024, nbumps=16, amp=0.01, width=0.05, gamma=GAMMA, cfl=0.5, nsteps=100) -> Problem:
    """Point-sampled density wave plus nbumps Gaussian bumps, U = V = 1, p = 1, periodic [0,2]^2."""
    rng = np.random.default_rng(seed)
    d = 2.0 / n
    xc = _centres(n, 0.0, d)[None, :]
    yc = _centres(n, 0.0, d)[:, None]
    rho = 1.0 + 0.2 * np.sin(np.pi * (xc + yc)) + _bump_field(n, rng, nbumps, amp, width)
    one = np.ones((n, n))
    W = _assemble(rho, one, one, one, gamma)
    return Problem("bumps", n, n, 0.0, 0.0, d, d, BC_PERIODIC, BC_PERIODIC, W, np.ones((n, n)),
                   flux=FLUX_LF, cfl=cfl, nsteps=nsteps, gamma=gamma, extra={"seed": seed})


def bumps_target(n, t, seed=1025, nbumps=16, amp=0.01, width=0.05) -> np.ndarray:
    """Target density of the adjoint loss: the wave advected to time t plus fresh seeded bumps."""
    rng = np.random.default_rng(seed)
    d = 2.0 / n
    xc = _centres(n, 0.0, d)[None, :]
    yc = _centres(n, 0.0, d)[:, None]
    return 1.0 + 0.2 * np.sin(np.pi * (xc + yc - 2.0 * t)) + _bump_field(n, rng, nbumps, amp, width)


# ------------------------------------------------------------------------------------------------
# Robustness problems of Section 4.3 (deterministic; the Mach number is the parameter).
# ------------------------------------------------------------------------------------------------

def problem_123(mach, n=100, gamma=GAMMA) -> Problem:
    """The 123 problem: (rho, u, p) = (1, -2, p0) on [0, 0.5) and (1, 2, p0) on [0.5, 1], two strong
    rarefactions leaving near-vacuum between them.  The reference Mach number |u| / sqrt(gamma p0 /
    rho) fixes p0 = rho u^2 / (gamma Ma^2).  n cells (ny = 1, dy = dx), free (transmissive)
    boundaries, final time 0.14."""
    d = 1.0 / n
    xc = _centres(n, 0.0, d)[None, :]
    rho = np.ones((1, n))
    u = np.where(xc < 0.5, -2.0, 2.0)
    p0 = 1.0 * 2.0 ** 2 / (gamma * mach ** 2)
    W = _assemble(rho, u, 0.0 * u, p0 * rho, gamma)
    return Problem("problem_123", n, 1, 0.0, 0.0, d, d, BC_TRANSMISSIVE, BC_TRANSMISSIVE, W, np.ones((1, n)),
                   cfl=0.5, gamma=gamma, extra={"mach": float(mach), "p0": p0, "t_end": 0.14})


def hurricane(mach, n=400, gamma=GAMMA, rho0=1.0, A=25.0) -> Problem:
    """Hurricane-like flow: (rho, u, v, p) = (rho0, v0 sin(theta), -v0 cos(theta), A rho0^gamma) on
    [-2,2]^2, theta the polar angle of (x, y), so the velocity is a rotation of speed |v0| about the
    origin (the paper writes theta = arctan(y/x); read as the polar angle).  Reference Mach number
    |v0| / c0 with c0 = sqrt(gamma A rho0^(gamma-1)).  Point values at the cell centres; dx = 4 / n
    (n = 400 gives the paper's 1/100), transmissive ("non-reflecting") boundaries; the test is
    survival over the first 50 steps."""
    d = 4.0 / n
    xc = _centres(n, -2.0, d)[None, :]
    yc = _centres(n, -2.0, d)[:, None]
    r = np.sqrt(xc * xc + yc * yc)
    c0 = math.sqrt(gamma * A * rho0 ** (gamma - 1.0))
    v0 = mach * c0
    rho = np.full((n, n), rho0)
    u = v0 * (yc / r) + 0.0 * xc   # v0 sin(theta)
    v = -v0 * (xc / r) + 0.0 * yc  # -v0 cos(theta)
    W = _assemble(rho, u, v, A * rho0 ** gamma * np.ones((n, n)), gamma)
    return Problem("hurricane", n, n, -2.0, -2.0, d, d, BC_TRANSMISSIVE, BC_TRANSMISSIVE, W, np.ones((n, n)),
                   cfl=0.5, nsteps=50, gamma=gamma, extra={"mach": float(mach), "v0": v0, "c0": c0})


def rarefaction2d(mach, n=400, gamma=GAMMA, A=1.5, q=0.6323) -> Problem:
    """Interaction of planar rarefaction waves on [0,1]^2 split at (0.5, 0.5):
    SW (1, -q, -q, 1.5), SE (rho, q, -q, A rho^gamma), NE (1, q, q, 1.5), NW (rho, -q, q, A rho^gamma)
    with q = 0.6323 and A = 1.5 (the NE state is garbled in the paper; read as (1, q, q, 1.5)).
    The reference Mach number sqrt(U^2 + V^2) / sqrt(gamma A rho^(gamma-1)) of the SE and NW states
    fixes rho = ((U^2 + V^2) / (gamma A Ma^2))^(1 / (gamma - 1)).  dx = 1 / n (n = 400 in the
    paper), free boundaries, final time 0.15."""
    d = 1.0 / n
    xc = _centres(n, 0.0, d)[None, :] + 0.0 * _centres(n, 0.0, d)[:, None]
    yc = _centres(n, 0.0, d)[:, None] + 0.0 * _centres(n, 0.0, d)[None, :]
    rho_q = ((2.0 * q * q) / (gamma * A * mach ** 2)) ** (1.0 / (gamma - 1.0))
    east, north = xc >= 0.5, yc >= 0.5
    diag = east == north  # SW and NE
    rho = np.where(diag, 1.0, rho_q)
    u = np.where(east, q, -q)
    v = np.where(north, q, -q)
    p = np.where(diag, 1.5, A * rho_q ** gamma)
    W = _assemble(rho, u, v, p, gamma)
    return Problem("rarefaction2d", n, n, 0.0, 0.0, d, d, BC_TRANSMISSIVE, BC_TRANSMISSIVE, W, np.ones((n, n)),
                   cfl=0.5, gamma=gamma, extra={"mach": float(mach), "rho": rho_q, "t_end": 0.15})


ROBUSTNESS = {"123": problem_123, "hurricane": hurricane, "rarefaction": rarefaction2d}
