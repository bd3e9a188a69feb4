"""Runs that stop at a final time (t_end) on the GPU against the oracle, through the C ABI: the last
step is shortened to end exactly on t_end, later steps are skipped (dt 0), for S2O4 (GKS, LF) and
SSP-RK3, with CFL and with fixed time steps, single grids and the batched form."""
import numpy as np
import pytest

import oracle as O
from paper_2402_10914_amd import workloads as WL

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _api():
    from paper_2402_10914_amd import api
    return api


def _rel_l1(a, b):
    """Parity measure: the larger of the relative L1 (sum|a - b| / sum|b|, per component) and a tenth
    of the per-cell relative maximum (max|a - b| / max|b|), max over components; a bound eps on it
    bounds the grid-wide sum by eps and every single cell by 10 eps, so that an error confined to a
    tile seam or a boundary row cannot hide in the sum."""
    if a.ndim == 2:
        a, b = a[None], b[None]
    return max(max(float(np.abs(a[c] - b[c]).sum() / max(np.abs(b[c]).sum(), 1e-300)),
                   0.1 * float(np.abs(a[c] - b[c]).max() / max(np.abs(b[c]).max(), 1e-300))) for c in range(a.shape[0]))


def _pair(pr, nsteps, **kw):
    api = _api()
    st = api.Stepper.for_problem(pr, api.Params(**kw), torch.float64)
    W = torch.tensor(pr.W, dtype=torch.float64, device="cuda")
    A = torch.tensor(pr.alpha, dtype=torch.float64, device="cuda")
    dth = torch.zeros(nsteps, dtype=torch.float64, device="cuda")
    t, fs = st.run(W, A, nsteps, dt_hist=dth)
    g = O.make_grid(pr.nx, pr.ny, pr.dx, pr.dy, pr.bc_x, pr.bc_y)
    Wo, Ao, to, dto, fso = O.run(pr.W, pr.alpha, g, O.make_params(**kw), nsteps)
    return (W.cpu().numpy(), A.cpu().numpy(), t, dth.cpu().numpy(), fs), (Wo, Ao, to, dto, fso)


@pytest.mark.parametrize("kw", [dict(flux=1, cfl=0.4), dict(flux=0, cfl=0.4),
                                dict(flux=0, cfl=0.4, time_scheme=1), dict(flux=1, cfl=0.4, time_limiter=1)])
def test_t_end_run_matches_oracle(kw):
    pr = WL.riemann4(48, 40, seed=7)
    (W, A, t, dth, fs), (Wo, Ao, to, dto, fso) = _pair(pr, 200, t_end=0.02, **kw)
    assert fs == -1 and fso == -1
    assert t == 0.02 and to == 0.02
    k = int(np.count_nonzero(dto))
    assert 0 < k < 200 and np.count_nonzero(dth) == k and np.all(dth[k:] == 0.0)
    np.testing.assert_allclose(dth, dto, rtol=1e-12)
    assert _rel_l1(W, Wo) <= 1e-12 and _rel_l1(A, Ao) <= 1e-12


def test_t_end_with_fixed_steps():
    pr = WL.density_wave(32)
    (W, A, t, dth, fs), (Wo, Ao, to, dto, fso) = _pair(pr, 20, flux=0, dt_fixed=0.007, t_end=0.05)
    assert t == 0.05 and to == 0.05
    np.testing.assert_allclose(dth[:7], 0.007, rtol=0, atol=0)
    assert dth[7] == dto[7] and 0 < dth[7] < 0.007 and np.all(dth[8:] == 0.0)
    assert _rel_l1(W, Wo) <= 1e-12


def test_t_end_batch_equals_loop_bitwise():
    api = _api()
    rng = np.random.default_rng(77)
    probs = [WL.riemann4(int(a), int(b), seed=[77, g]) for g, (a, b) in enumerate(rng.integers(8, 64, (6, 2)))]
    params = api.Params(flux=api.FLUX_GKS, cfl=0.4, time_limiter=1, t_end=0.03)
    b = api.Batch([(p.nx, p.ny, p.dx, p.dy, p.bc_x, p.bc_y) for p in probs], params, torch.float64, 0)
    W, A = b.pack([p.W for p in probs], [p.alpha for p in probs])
    ts, fs = b.run(W, A, 120, use_graph=True)
    assert all(f == -1 for f in fs) and all(t == 0.03 for t in ts)
    for p, (w, a) in zip(probs, b.unpack(W, A)):
        st = api.Stepper.for_problem(p, params, torch.float64)
        Wl = torch.tensor(p.W, dtype=torch.float64, device="cuda")
        Al = torch.tensor(p.alpha, dtype=torch.float64, device="cuda")
        t, f = st.run(Wl, Al, 120)
        assert t == 0.03 and f == -1
        assert torch.equal(w, Wl) and torch.equal(a, Al)
