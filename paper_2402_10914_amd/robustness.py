"""Robustness sweeps of Section 4.3 (Tables 5-7): the largest reference Mach number at which a
scheme runs a problem to its end without meeting a non-physical state (rho <= 0, p <= 0 or a
non-finite value), found by a bisection in which every round advances a set of candidate Mach
numbers together as one batch of independent grids (one captured hipGraph launch).

Schemes, the paper's two solvers: ``gks`` = S2O4 with the gas-kinetic flux and the non-linear
time limiter (eqs. (21), (27)-(29)); ``lf`` = SSP-RK3 with the Lax-Friedrichs flux (eq. (32)).
Reconstructions: ``weno_ao`` (DF threshold 0: the switch never engages), ``hybrid`` (threshold 0.5,
the switch of eq. (42) as printed: the largest DF value of the three cells below the threshold) and
``hybrid_min`` (the same with the smallest of the three) and ``hybrid_own`` (the cell's own DF
value).  Initial DF: ``one`` (alpha^0 = 1) or
``initial`` (the DF product of the initial state's own Gauss-point values, one evaluation of the
operator before the first step).  CFL 0.5, as the paper uses for these problems.

    python -m paper_2402_10914_amd.robustness --problems 123,hurricane,rarefaction
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import workloads as WL

SOLVERS = ("gks", "lf")
RECONS = ("weno_ao", "hybrid", "hybrid_min", "hybrid_own")
ALPHA0 = ("one", "initial")


def solver_params(solver: str, recon: str, t_end: float = 0.0, **ablation):
    """Parameters of one configuration; `ablation` passes further options (componentwise, df_stage)."""
    from .api import FLUX_GKS, FLUX_LF, TIME_S2O4, TIME_SSPRK3, Params
    thres, rule = {"hybrid": (0.5, 0), "hybrid_min": (0.5, 1), "hybrid_own": (0.5, 2), "weno_ao": (0.0, 0)}[recon]
    if solver == "gks":
        return Params(flux=FLUX_GKS, cfl=0.5, alpha_thres=thres, switch_rule=rule, time_limiter=1,
                      time_scheme=TIME_S2O4, t_end=t_end, **ablation)
    if solver == "lf":
        return Params(flux=FLUX_LF, cfl=0.5, alpha_thres=thres, switch_rule=rule, time_scheme=TIME_SSPRK3,
                      t_end=t_end, **ablation)
    raise ValueError(f"unknown solver {solver!r}")


def initial_alpha(pr, params, dtype):
    """alpha^0 from the initial state: the DF product of the Gauss-point values of one evaluation of
    the spatial operator (with alpha = 1) on the GPU."""
    import torch
    from .api import Stepper
    st = Stepper.for_problem(pr, params, dtype)
    W = torch.tensor(pr.W, dtype=dtype, device="cuda")
    A = torch.ones((pr.ny, pr.nx), dtype=dtype, device="cuda")
    smax, _ = st.max_speed(W)
    _, _, an = st.rhs(W, A, pr.cfl / smax, want_alpha=True)
    return an.double().cpu().numpy()


def max_signal_speed(pr, dtype=None) -> float:
    """The CFL reduction of the initial state on the GPU (the library's dfw_max_speed)."""
    import torch
    from .api import Params, Stepper
    dtype = torch.float64 if dtype is None else dtype
    st = Stepper.for_problem(pr, Params(gamma=pr.gamma), dtype)
    smax, _ = st.max_speed(torch.tensor(pr.W, dtype=dtype, device="cuda"))
    return smax


def step_cap(pr, smax: float) -> int:
    """Upper bound on the steps to the problem's end, given the initial state's maximum signal speed
    over the cell size (the CFL reduction): four times the steps that speed would need (the speeds
    of these flows grow by well under that factor)."""
    t_end = pr.extra.get("t_end", 0.0)
    if t_end <= 0.0:
        return pr.nsteps
    dt0 = pr.cfl / smax
    return int(math.ceil(4.0 * t_end / dt0)) + 20


def run_batch(problem: str, machs, solver: str, recon: str, n: int | None = None, dtype=None, alpha0: str = "one",
              ablation: dict | None = None):
    """Runs the problem at every Mach number of `machs` as one batch (one captured hipGraph) to its
    end; returns (final time per run, failing step per run or -1, step cap)."""
    import torch
    from .api import Batch
    dtype = torch.float64 if dtype is None else dtype
    make = WL.ROBUSTNESS[problem]
    probs = [make(float(m)) if n is None else make(float(m), n=n) for m in machs]
    t_end = probs[0].extra.get("t_end", 0.0)
    params = solver_params(solver, recon, t_end, **(ablation or {}))
    if alpha0 == "initial":
        for p in probs:
            p.alpha = initial_alpha(p, params, dtype)
    elif alpha0 != "one":
        raise ValueError(f"unknown alpha0 {alpha0!r}")
    b = Batch([(p.nx, p.ny, p.dx, p.dy, p.bc_x, p.bc_y) for p in probs], params, dtype, 0)
    W, A = b.pack([p.W for p in probs], [p.alpha for p in probs])
    nsteps = max(step_cap(p, max_signal_speed(p, dtype)) for p in probs)
    t, fs = b.run(W, A, nsteps, use_graph=True)
    return t, fs, nsteps


def survives(problem: str, machs, solver: str, recon: str, n: int | None = None, dtype=None, alpha0: str = "one",
             ablation: dict | None = None):
    """Runs the problem at every Mach number of `machs` as one batch; returns [bool] (survived)."""
    t, fs, nsteps = run_batch(problem, machs, solver, recon, n, dtype, alpha0, ablation)
    t_end = WL.ROBUSTNESS[problem](float(machs[0]), **({} if n is None else {"n": n})).extra.get("t_end", 0.0)
    out = []
    for ti, f in zip(t, fs):
        if f != -1:
            out.append(False)
        elif t_end > 0.0 and ti != t_end:
            raise RuntimeError(f"{problem}: t_end not reached in {nsteps} steps (t = {ti})")
        else:
            out.append(True)
    return out


def max_mach(problem: str, solver: str, recon: str, lo: float = 1.0, hi: float = 200.0, k: int = 16,
             rtol: float = 0.01, runner=None, **kw) -> dict:
    """Bisection for the survival boundary in [lo, hi]: each round evaluates k Mach numbers spaced
    geometrically strictly inside the bracket; the bracket becomes (largest survivor below the first
    failure, first failure).  Stops when hi / lo <= 1 + rtol.  `runner(machs) -> [bool]` defaults to
    the GPU batch (`survives`).  Returns {"max_mach": lo, "first_fail": hi, ...}; max_mach is None
    when lo already fails and first_fail None when hi survives."""
    run = runner or (lambda ms: survives(problem, ms, solver, recon, **kw))
    evals, rounds = 2, 0
    ok_lo, ok_hi = run([lo, hi])
    res = dict(problem=problem, solver=solver, recon=recon, rtol=rtol, k=k)
    if not ok_lo:
        return dict(res, max_mach=None, first_fail=lo, rounds=0, evaluations=evals)
    if ok_hi:
        return dict(res, max_mach=hi, first_fail=None, rounds=0, evaluations=evals)
    while hi / lo > 1.0 + rtol:
        pts = np.geomspace(lo, hi, k + 2)[1:-1]
        ok = run([float(p) for p in pts])
        evals += len(pts)
        rounds += 1
        fails = [i for i, o in enumerate(ok) if not o]
        if not fails:
            lo = float(pts[-1])
        else:
            j = fails[0]
            hi = float(pts[j])
            if j > 0:
                lo = float(pts[j - 1])
    return dict(res, max_mach=lo, first_fail=hi, rounds=rounds, evaluations=evals)


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--problems", default="123,hurricane,rarefaction")
    ap.add_argument("--solvers", default="gks,lf")
    ap.add_argument("--recons", default="weno_ao,hybrid,hybrid_min,hybrid_own")
    ap.add_argument("--alpha0", default="one,initial", help="initial DF of the hybrid runs")
    ap.add_argument("--k", type=int, default=16)
    ap.add_argument("--rtol", type=float, default=0.01)
    ap.add_argument("--lo", type=float, default=1.0)
    ap.add_argument("--hi", type=float, default=200.0)
    ap.add_argument("--componentwise", type=int, default=0, help="1: component-wise reconstruction (ablation)")
    ap.add_argument("--df-stage", type=int, default=0, help="1: DF from the first stage (ablation)")
    a = ap.parse_args(argv)
    ablation = dict(componentwise=a.componentwise, df_stage=a.df_stage)
    for prob in a.problems.split(","):
        for solver in a.solvers.split(","):
            for recon in a.recons.split(","):
                for alpha0 in (a.alpha0.split(",") if recon != "weno_ao" else ["one"]):
                    t0 = time.time()
                    r = max_mach(prob, solver, recon, lo=a.lo, hi=a.hi, k=a.k, rtol=a.rtol, alpha0=alpha0,
                                 ablation=ablation)
                    r["alpha0"] = alpha0
                    r.update(ablation)
                    r["seconds"] = round(time.time() - t0, 2)
                    print(json.dumps(r), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
