"""The batched survival runner of the Section 4.3 robustness sweeps on the GPU: its verdicts for the 123
problem equal those of oracle runs of the same configurations (Mach numbers chosen away from the
survival boundaries, where a rounding difference cannot flip a verdict), and one bisection brackets
a boundary to the requested tolerance."""
import numpy as np
import pytest

import oracle as O
from paper_2402_10914_amd import workloads as WL

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _oracle_survives(mach, solver, recon, alpha0):
    from paper_2402_10914_amd import robustness as R
    pr = WL.problem_123(mach)
    p = R.solver_params(solver, recon, pr.extra["t_end"])
    P = O.make_params(flux=p.flux, cfl=p.cfl, alpha_thres=p.alpha_thres, switch_rule=p.switch_rule,
                      time_limiter=p.time_limiter, time_scheme=p.time_scheme, t_end=p.t_end)
    g = O.make_grid(pr.nx, pr.ny, pr.dx, pr.dy, pr.bc_x, pr.bc_y)
    a0 = pr.alpha
    if alpha0 == "initial":
        _, _, a0 = O.rhs(pr.W, pr.alpha, g, P, pr.cfl / O.max_speed(pr.W, g, P)[0], want_alpha=True)
    _, _, t, _, fs = O.run(pr.W, a0, g, P, R.step_cap(pr))
    return fs == -1 and t == p.t_end


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
