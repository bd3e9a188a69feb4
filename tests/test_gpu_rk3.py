"""SSP-RK3 (Section 2.3, eq. (32)) with the LF flux on the GPU against the oracle, through the C ABI:
Riemann data and the density wave in FP64 (rel-L1 <= 1e-12), FP32 (<= 1e-5), ragged and degenerate
grids, periodic conservation, bitwise determinism, transpose symmetry, and the batched form bitwise
equal to the per-grid loop."""
import numpy as np
import pytest

import oracle as O
from paper_2402_10914_amd import workloads as WL

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL64, TOL32 = 1e-12, 1e-5


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


def _gpu_run(pr, nsteps, dtype=torch.float64, cfl=0.4, W0=None):
    api = _api()
    st = api.Stepper.for_problem(pr, api.Params(flux=api.FLUX_LF, cfl=cfl, time_scheme=api.TIME_SSPRK3), dtype)
    W = torch.tensor(pr.W if W0 is None else W0, dtype=dtype, device="cuda")
    A = torch.tensor(pr.alpha, dtype=dtype, device="cuda")
    dth = torch.zeros(max(nsteps, 1), dtype=torch.float64, device="cuda")
    t, fs = st.run(W, A, nsteps, dt_hist=dth)
    return W.double().cpu().numpy(), A.double().cpu().numpy(), t, dth.cpu().numpy()[:nsteps], fs


def _oracle_run(pr, nsteps, cfl=0.4):
    g = O.make_grid(pr.nx, pr.ny, pr.dx, pr.dy, pr.bc_x, pr.bc_y)
    return O.run(pr.W, pr.alpha, g, O.make_params(flux=O.FLUX_LF, cfl=cfl, time_scheme=O.TIME_SSPRK3), nsteps)


@pytest.mark.parametrize("nx,ny,seed", [(48, 40, 48), (33, 17, 11)])
def test_rk3_riemann_run_matches_oracle(nx, ny, seed):
    pr = WL.riemann4(nx, ny, seed=seed)
    W, A, t, dth, fs = _gpu_run(pr, 20)
    Wo, Ao, to, dto, fso = _oracle_run(pr, 20)
    assert fs == -1 and fso == -1
    assert _rel_l1(W, Wo) <= TOL64
    assert _rel_l1(A, Ao) <= TOL64
    np.testing.assert_allclose(dth, dto, rtol=1e-12)
    assert abs(t - to) <= 1e-12 * to


def test_rk3_density_wave_matches_oracle_and_exact_solution():
    pr = WL.density_wave(64)
    W, A, t, dth, fs = _gpu_run(pr, 20, cfl=0.5)
    Wo, Ao, to, dto, fso = _oracle_run(pr, 20, cfl=0.5)
    assert fs == -1 and fso == -1
    assert _rel_l1(W, Wo) <= TOL64
    assert np.all(np.abs(A - 1.0) <= 1e-12)
    err = np.abs(W[0] - WL.density_wave_avg(64, 64, t=t)).mean()
    assert err < 2e-5, err


def test_rk3_fp32_matches_oracle():
    pr = WL.riemann4(40, 36, seed=36)
    W, A, _, _, fs = _gpu_run(pr, 10, dtype=torch.float32)
    Wo, Ao, _, _, fso = _oracle_run(pr, 10)
    assert fs == -1 and fso == -1
    assert _rel_l1(W, Wo) <= TOL32
    print(f"ssprk3 fp32: W {_rel_l1(W, Wo):.3e} alpha {_rel_l1(A, Ao):.3e}", flush=True)
    assert _rel_l1(A, Ao) <= TOL32


@pytest.mark.parametrize("nx,ny", [(1, 9), (30, 1), (5, 40), (64, 3), (17, 29)])
def test_rk3_ragged_and_degenerate_grids(nx, ny):
    pr = WL.riemann4(nx, ny, seed=nx * 100 + ny)
    W, A, _, dth, fs = _gpu_run(pr, 3)
    Wo, Ao, _, dto, fso = _oracle_run(pr, 3)
    assert fs == fso
    assert _rel_l1(W, Wo) <= TOL64
    assert _rel_l1(A, Ao) <= TOL64
    np.testing.assert_allclose(dth, dto, rtol=1e-12)


def test_rk3_periodic_conservation_determinism_and_symmetry():
    pr = WL.circles(64, seed=7, ncirc=6)
    W, _, _, _, fs = _gpu_run(pr, 10)
    assert fs == -1
    s0, s1 = pr.W.sum(axis=(1, 2)), W.sum(axis=(1, 2))
    assert np.all(np.abs(s1 - s0) <= 1e-13 * np.abs(pr.W).sum(axis=(1, 2)))
    pr = WL.riemann4(36, 36, seed=21)
    A1, a1, _, _, _ = _gpu_run(pr, 8)
    A2, a2, _, _, _ = _gpu_run(pr, 8)
    assert np.array_equal(A1, A2) and np.array_equal(a1, a2)
    Wt = np.stack([pr.W[0].T, pr.W[2].T, pr.W[1].T, pr.W[3].T]).copy()
    prt = WL.riemann4(36, 36, seed=21)
    prt.alpha = pr.alpha.T.copy()
    B, b, _, _, _ = _gpu_run(prt, 8, W0=Wt)
    Bt = np.stack([B[0].T, B[2].T, B[1].T, B[3].T])
    # the S2O4 kernels are transpose-symmetric bit for bit; the derivative-free interface kernel of
    # these stages gives x- and y-faces results that differ in the last bit, so rounding level here
    np.testing.assert_allclose(Bt, A1, rtol=0, atol=1e-13 * np.abs(A1).max())
    np.testing.assert_allclose(b.T, a1, rtol=0, atol=1e-13)


def test_rk3_batch_equals_loop_bitwise():
    api = _api()
    rng = np.random.default_rng(31)
    probs = [WL.riemann4(int(a), int(b), seed=[31, g]) for g, (a, b) in enumerate(rng.integers(6, 70, (7, 2)))]
    params = api.Params(flux=api.FLUX_LF, cfl=0.4, time_scheme=api.TIME_SSPRK3)
    b = api.Batch([(p.nx, p.ny, p.dx, p.dy, p.bc_x, p.bc_y) for p in probs], params, torch.float64, 0)
    W, A = b.pack([p.W for p in probs], [p.alpha for p in probs])
    _, fs = b.run(W, A, 6, use_graph=True)
    for p, (w, a), f in zip(probs, b.unpack(W, A), fs):
        Wl, Al, _, _, fl = _gpu_run(p, 6)
        assert f == fl
        assert np.array_equal(w.cpu().numpy(), Wl) and np.array_equal(a.cpu().numpy(), Al)


def test_rk3_rejects_gks_and_the_time_limiter():
    api = _api()
    pr = WL.riemann4(16, 16, seed=1)
    for kw in (dict(flux=api.FLUX_GKS), dict(flux=api.FLUX_LF, time_limiter=1)):
        st = api.Stepper.for_problem(pr, api.Params(cfl=0.4, time_scheme=api.TIME_SSPRK3, **kw), torch.float64)
        W = torch.tensor(pr.W, dtype=torch.float64, device="cuda")
        A = torch.tensor(pr.alpha, dtype=torch.float64, device="cuda")
        with pytest.raises(api.DFWError):
            st.run(W, A, 1)
