"""The robustness problems of Section 4.3 (Tables 5-7) on the GPU against the oracle.

* 123 problem: the batched survival runner's verdicts equal those of oracle runs of the same
  configurations (Mach numbers chosen away from the survival boundaries, where a rounding difference
  cannot flip a verdict), and one bisection brackets a boundary to the requested tolerance.
* Hurricane-like flow and interaction of planar rarefactions (on 40x40 grids, so the oracle finishes
  in seconds): the first steps of every solver / reconstruction against the oracle cell by cell, and
  the step at which each whole run fails (or that it survives) equal to the oracle's at Mach numbers
  on both sides of the survival boundaries."""
import numpy as np
import pytest

import oracle as O
from paper_2402_10914_amd import workloads as WL

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _oracle_setup(problem, mach, solver, recon, alpha0, n=None):
    from paper_2402_10914_amd import robustness as R
    pr = WL.ROBUSTNESS[problem](mach) if n is None else WL.ROBUSTNESS[problem](mach, n=n)
    p = R.solver_params(solver, recon, pr.extra.get("t_end", 0.0))
    P = O.make_params(flux=p.flux, cfl=p.cfl, alpha_thres=p.alpha_thres, switch_rule=p.switch_rule,
                      time_limiter=p.time_limiter, time_scheme=p.time_scheme, t_end=p.t_end)
    g = O.make_grid(pr.nx, pr.ny, pr.dx, pr.dy, pr.bc_x, pr.bc_y)
    smax = O.max_speed(pr.W, g, P)[0]
    a0 = pr.alpha
    if alpha0 == "initial":
        _, _, a0 = O.rhs(pr.W, pr.alpha, g, P, pr.cfl / smax, want_alpha=True)
    return pr, p, P, g, a0, R.step_cap(pr, smax)


def _oracle_run(problem, mach, solver, recon, alpha0, n=None):
    pr, p, P, g, a0, cap = _oracle_setup(problem, mach, solver, recon, alpha0, n)
    _, _, t, _, fs = O.run(pr.W, a0, g, P, cap)
    return t, fs, p.t_end


def _oracle_survives(mach, solver, recon, alpha0):
    t, fs, t_end = _oracle_run("123", mach, solver, recon, alpha0)
    return fs == -1 and t == t_end


@pytest.mark.parametrize("solver", ["gks", "lf"])
def test_batched_survival_matches_oracle(solver):
    from paper_2402_10914_amd import robustness as R
    machs = [1.5, 3.0, 10.0]
    for recon, alpha0 in (("weno_ao", "one"), ("hybrid", "one"), ("hybrid_own", "initial")):
        got = R.survives("123", machs, solver, recon, alpha0=alpha0)
        want = [_oracle_survives(m, solver, recon, alpha0) for m in machs]
        assert got == want, (recon, got, want)
    assert R.survives("123", [1.5, 3.0], solver, "weno_ao") == [True, False]
    assert R.survives("123", [10.0], solver, "hybrid_own", alpha0="initial") == [True]


def test_bisection_on_the_gpu():
    from paper_2402_10914_amd import robustness as R
    r = R.max_mach("123", "lf", "weno_ao", lo=1.0, hi=4.0, k=8, rtol=0.02)
    assert r["max_mach"] is not None and r["first_fail"] is not None
    assert 1.0 <= r["max_mach"] < r["first_fail"] <= 4.0 and r["first_fail"] / r["max_mach"] <= 1.02
    assert R.survives("123", [r["max_mach"]], "lf", "weno_ao") == [True]
    assert R.survives("123", [r["first_fail"]], "lf", "weno_ao") == [False]


_CONFIGS = [("weno_ao", "one"), ("hybrid", "one"), ("hybrid_own", "initial")]


@pytest.mark.parametrize("recon,alpha0", _CONFIGS)
@pytest.mark.parametrize("solver", ["gks", "lf"])
@pytest.mark.parametrize("problem", ["hurricane", "rarefaction"])
def test_robustness_problem_first_steps_match_oracle(problem, solver, recon, alpha0):
    """Mach 1.1 on a 40x40 grid (every configuration survives): the state and DF after the first
    steps, every cell, GPU against oracle.  GKS runs with the time limiter, whose step map
    amplifies rounding near jumps, so its comparison stops after four steps."""
    from paper_2402_10914_amd import api
    from paper_2402_10914_amd import robustness as R
    pr, p, P, g, a0, _ = _oracle_setup(problem, 1.1, solver, recon, alpha0, n=40)
    steps = 4 if solver == "gks" else 10
    Wo, Ao, to, dto, fso = O.run(pr.W, a0, g, P, steps)
    assert fso == -1
    st = api.Stepper.for_problem(pr, p)
    W = torch.tensor(pr.W, device="cuda")
    A = torch.tensor(a0 if alpha0 == "one" else R.initial_alpha(pr, p, torch.float64), device="cuda")
    np.testing.assert_allclose(A.cpu().numpy(), a0, rtol=0, atol=1e-13)
    dth = torch.zeros(steps, dtype=torch.float64, device="cuda")
    t, fs = st.run(W, A, steps, dt_hist=dth)
    assert fs == -1
    Wg, Ag = W.cpu().numpy(), A.cpu().numpy()
    for c in range(4):
        assert np.abs(Wg[c] - Wo[c]).sum() / np.abs(Wo[c]).sum() <= 1e-12, c
    assert np.abs(Wg - Wo).max() <= 1e-11 * np.abs(Wo).max()
    assert np.abs(Ag - Ao).sum() / np.abs(Ao).sum() <= 1e-12
    assert np.abs(Ag - Ao).max() <= 1e-11
    np.testing.assert_allclose(dth.cpu().numpy(), dto, rtol=1e-12)
    assert abs(t - to) <= 1e-12 * to


# (problem, solver) -> Mach numbers on both sides of the 40x40 survival boundaries of every
# configuration of _CONFIGS (oracle: survives at 1.1; fails within the first steps at 12)
_MACHS = {("hurricane", "gks"): [1.1, 3.0, 12.0], ("hurricane", "lf"): [1.1, 2.0, 12.0],
          ("rarefaction", "gks"): [1.1, 3.0, 12.0], ("rarefaction", "lf"): [1.1, 3.0, 12.0]}


@pytest.mark.parametrize("solver", ["gks", "lf"])
@pytest.mark.parametrize("problem", ["hurricane", "rarefaction"])
def test_robustness_problem_fail_steps_match_oracle(problem, solver):
    """Whole runs to the problem's end (hurricane: 50 steps; rarefactions: t = 0.15) in the batched
    runner on 40x40 grids: the step at which each run meets a non-physical state, or its survival to
    the end time, equals the oracle's for every configuration."""
    from paper_2402_10914_amd import robustness as R
    machs = _MACHS[(problem, solver)]
    for recon, alpha0 in _CONFIGS:
        t, fs, _ = R.run_batch(problem, machs, solver, recon, n=40, alpha0=alpha0)
        want = [_oracle_run(problem, m, solver, recon, alpha0, n=40) for m in machs]
        assert [f for f in fs] == [w[1] for w in want], (recon, fs, want)
        for ti, (to, fo, t_end) in zip(t, want):
            if fo == -1 and t_end > 0.0:
                assert ti == t_end and to == t_end
        assert fs[0] == -1 and fs[-1] != -1
