"""Host logic of the Section 4.3 robustness sweeps (CPU): the initial states carry the requested
reference Mach numbers, and the batched bisection finds the survival boundary of a synthetic
survival rule."""
import math

import numpy as np
import pytest

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


def test_step_cap_covers_the_run():
    pr = WL.problem_123(10.0)
    dt0 = 0.5 * pr.dx / (2.0 + 2.0 / 10.0)
    assert R.step_cap(pr) >= 4 * 0.14 / dt0
    assert R.step_cap(WL.hurricane(3.0, n=40)) == 50
    with pytest.raises(ValueError):
        R.solver_params("roe", "hybrid")
