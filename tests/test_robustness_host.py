"""Host logic of the Section 4.3 robustness sweeps (CPU): the initial states carry the requested
reference Mach numbers, and the batched bisection finds the survival boundary of a synthetic
survival rule."""
import math

import numpy as np
import pytest

import oracle as O

from paper_2402_10914_amd import robustness as R
from paper_2402_10914_amd import workloads as WL

GAMMA = 1.4


def _prim(pr):
    W = pr.W
    rho = W[0]
    u, v = W[1] / rho, W[2] / rho
    p = (GAMMA - 1.0) * (W[3] - 0.5 * rho * (u * u + v * v))
    return rho, u, v, p


@pytest.mark.parametrize("mach", [2.0, 31.5, 84.1])
def test_problem_123_states(mach):
    pr = WL.problem_123(mach)
    rho, u, v, p = _prim(pr)
    assert pr.nx == 100 and pr.ny == 1 and pr.extra["t_end"] == 0.14
    assert np.all(rho == 1.0) and np.all(v == 0.0)
    assert np.all(u[:, :50] == -2.0) and np.all(u[:, 50:] == 2.0)
    c = np.sqrt(GAMMA * p / rho)
    np.testing.assert_allclose(np.abs(u) / c, mach, rtol=1e-13)


@pytest.mark.parametrize("mach", [1.5, 16.0])
def test_hurricane_states(mach):
    pr = WL.hurricane(mach, n=40)
    rho, u, v, p = _prim(pr)
    d = 4.0 / 40
    xc = -2.0 + (np.arange(40) + 0.5) * d
    X, Y = np.meshgrid(xc, xc)
    assert pr.dx == pytest.approx(d) and pr.nsteps == 50
    np.testing.assert_allclose(u * X + v * Y, 0.0, atol=1e-12 * mach)       # rotation about the origin
    np.testing.assert_allclose(u * Y - v * X, pr.extra["v0"] * np.hypot(X, Y), rtol=1e-13)  # clockwise, |v| = v0
    np.testing.assert_allclose(p, 25.0, rtol=1e-12)
    np.testing.assert_allclose(np.hypot(u, v) / np.sqrt(GAMMA * p / rho), mach, rtol=1e-12)


@pytest.mark.parametrize("mach", [1.8, 24.8])
def test_rarefaction2d_states(mach):
    pr = WL.rarefaction2d(mach, n=40)
    rho, u, v, p = _prim(pr)
    q = 0.6323
    sw, se, ne, nw = (np.s_[:20, :20], np.s_[:20, 20:], np.s_[20:, 20:], np.s_[20:, :20])
    for sl, su, sv in ((sw, -q, -q), (se, q, -q), (ne, q, q), (nw, -q, q)):
        np.testing.assert_allclose(u[sl], su, rtol=1e-13)
        np.testing.assert_allclose(v[sl], sv, rtol=1e-13)
    for sl in (sw, ne):
        np.testing.assert_allclose(rho[sl], 1.0, rtol=1e-14)
        np.testing.assert_allclose(p[sl], 1.5, rtol=1e-13)
    for sl in (se, nw):
        np.testing.assert_allclose(p[sl], 1.5 * rho[sl] ** GAMMA, rtol=1e-11)   # isentropic, A = 1.5
        ma = np.hypot(u[sl], v[sl]) / np.sqrt(GAMMA * 1.5 * rho[sl] ** (GAMMA - 1.0))
        np.testing.assert_allclose(ma, mach, rtol=1e-12)


@pytest.mark.parametrize("threshold", [1.7, 17.3, 150.0])
def test_bisection_brackets_the_survival_boundary(threshold):
    calls = []

    def runner(ms):
        calls.append(len(ms))
        return [m < threshold for m in ms]

    r = R.max_mach("123", "gks", "hybrid", lo=1.0, hi=200.0, k=16, rtol=0.01, runner=runner)
    assert r["max_mach"] < threshold <= r["first_fail"]
    assert r["first_fail"] / r["max_mach"] <= 1.01
    assert r["evaluations"] == sum(calls) and max(calls) <= 16
    assert r["rounds"] <= 3   # log(200) / log(17)^3 < log(1.01)


def test_bisection_open_ends():
    r = R.max_mach("123", "lf", "weno_ao", lo=2.0, hi=50.0, runner=lambda ms: [False] * len(ms))
    assert r["max_mach"] is None and r["first_fail"] == 2.0
    r = R.max_mach("123", "lf", "weno_ao", lo=2.0, hi=50.0, runner=lambda ms: [True] * len(ms))
    assert r["max_mach"] == 50.0 and r["first_fail"] is None


def _oracle_smax(pr):
    g = O.make_grid(pr.nx, pr.ny, pr.dx, pr.dy, pr.bc_x, pr.bc_y)
    return O.max_speed(pr.W, g, O.make_params(gamma=pr.gamma))[0]


def test_step_cap_covers_the_run():
    pr = WL.problem_123(10.0)
    dt0 = 0.5 * pr.dx / (2.0 + 2.0 / 10.0)
    assert R.step_cap(pr, _oracle_smax(pr)) >= 4 * 0.14 / dt0
    hur = WL.hurricane(3.0, n=40)
    assert R.step_cap(hur, _oracle_smax(hur)) == 50
    with pytest.raises(ValueError):
        R.solver_params("roe", "hybrid")


def _switch_counts(problem, mach, solver, n=None, steps=30):
    """Oracle run with the hybrid switch as printed (eq. (42)), one step at a time: per completed
    step the number of cells whose own DF is below the threshold and the number of (cell, direction)
    pairs meeting the printed condition (the DF of the cell and both neighbours along the direction
    below the threshold); stops at the failing step."""
    pr = WL.ROBUSTNESS[problem](mach) if n is None else WL.ROBUSTNESS[problem](mach, n=n)
    p = R.solver_params(solver, "hybrid", pr.extra.get("t_end", 0.0))
    P = O.make_params(flux=p.flux, cfl=p.cfl, alpha_thres=p.alpha_thres, switch_rule=p.switch_rule,
                      time_limiter=p.time_limiter, time_scheme=p.time_scheme, t_end=p.t_end)
    g = O.make_grid(pr.nx, pr.ny, pr.dx, pr.dy, pr.bc_x, pr.bc_y)
    W, a = pr.W, pr.alpha
    out = []
    for _ in range(steps):
        W, a, _, _, fs = O.run(W, a, g, P, 1)
        if fs != -1:
            return out, True
        pad = np.pad(a, 1, mode="edge")  # transmissive boundaries
        trip = 0
        for ax in ((0, 1), (1, 0)):
            if a.shape[1 if ax[1] else 0] == 1:
                continue
            nb = [pad[1 + dj:1 + dj + a.shape[0], 1 + di:1 + di + a.shape[1]] for dj, di in ((-ax[0], -ax[1]), (0, 0), (ax[0], ax[1]))]
            trip += int((np.maximum(np.maximum(nb[0], nb[1]), nb[2]) < 0.5).sum())
        out.append((int((a < 0.5).sum()), trip))
    return out, False


def test_printed_switch_stays_off_at_isolated_jumps():
    """Finding behind reading R31 (Section 4.3, Table 5): on the 123 problem the DF drops below the
    threshold in the two cells beside the central jump only, so the printed condition (three
    consecutive cells below 0.5) never holds and the hybrid run equals WENO-AO up to its failure;
    on the planar rarefactions the low-DF zone is wider than two cells and the condition holds."""
    for solver in ("gks", "lf"):
        counts, failed = _switch_counts("123", 3.0, solver)
        assert failed and counts
        assert counts[0][0] == 2
        assert all(trip == 0 for _, trip in counts)
    counts, failed = _switch_counts("rarefaction", 3.0, "lf", n=100)
    assert counts and counts[0][1] > 0
