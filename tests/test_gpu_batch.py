"""Batched ragged grids (one launch per kernel for all grids, one hipGraph replay for the rollout):
bitwise equal to the per-grid loop, to the ungraphed batch and across tile shapes and sweep
orders; parity with the oracle on sampled grids; per-grid failure isolation; the full 256-grid
configuration against the per-grid loop."""
import numpy as np
import pytest

import oracle as O
from paper_2402_10914_amd import workloads as WL

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _api():
    from paper_2402_10914_amd import api
    return api


def _small_batch(n=10, seed=77, lo=5, hi=70):
    rng = np.random.default_rng(seed)
    probs = []
    for g in range(n):
        nx, ny = (int(x) for x in rng.integers(lo, hi, 2))
        if g % 3 == 0:
            probs.append(WL.density_wave(nx, ny))
        else:
            probs.append(WL.riemann4(nx, ny, seed=[seed, g]))
    probs.append(WL.riemann4(1, 13, seed=3))  # degenerate strips
    probs.append(WL.riemann4(17, 1, seed=4))
    return probs


def _grids(probs):
    return [(p.nx, p.ny, p.dx, p.dy, p.bc_x, p.bc_y) for p in probs]


def _loop(probs, params, nsteps, dtype=torch.float64):
    api = _api()
    outs = []
    for p in probs:
        st = api.Stepper.for_problem(p, params, dtype)
        W = torch.tensor(p.W, dtype=dtype, device="cuda")
        A = torch.tensor(p.alpha, dtype=dtype, device="cuda")
        dth = torch.zeros(max(nsteps, 1), dtype=torch.float64, device="cuda")
        t, fs = st.run(W, A, nsteps, dt_hist=dth)
        outs.append((W.cpu().numpy(), A.cpu().numpy(), t, fs, dth.cpu().numpy()[:nsteps]))
    return outs


def _batched(probs, params, nsteps, dtype=torch.float64, order=0, use_graph=True, reps=1):
    api = _api()
    b = api.Batch(_grids(probs), params, dtype, order)
    W0, A0 = b.pack([p.W for p in probs], [p.alpha for p in probs])
    dth = torch.zeros(len(probs) * max(nsteps, 1), dtype=torch.float64, device="cuda")
    W, A = W0.clone(), A0.clone()
    for _ in range(reps):  # same buffers: the second run replays the captured graph
        W.copy_(W0)
        A.copy_(A0)
        t, fs = b.run(W, A, nsteps, use_graph=use_graph, dt_hist=dth)
    views = b.unpack(W, A)
    dh = dth.cpu().numpy().reshape(len(probs), -1)
    return [(w.cpu().numpy(), a.cpu().numpy(), t[g], fs[g], dh[g, :nsteps]) for g, (w, a) in enumerate(views)]


def _same(x, y):
    for (w1, a1, t1, f1, d1), (w2, a2, t2, f2, d2) in zip(x, y):
        assert np.array_equal(w1, w2, equal_nan=True) and np.array_equal(a1, a2, equal_nan=True)
        assert t1 == t2 and f1 == f2 and np.array_equal(d1, d2)


@pytest.mark.parametrize("flux", [0, 1])
def test_batch_equals_loop_bitwise(flux):
    probs = _small_batch()
    api = _api()
    params = api.Params(flux=flux, cfl=0.4)
    ref = _loop(probs, params, 12)
    _same(_batched(probs, params, 12, use_graph=True, reps=2), ref)  # capture, then a replay
    _same(_batched(probs, params, 12, use_graph=False), ref)


def test_batch_fp32_equals_loop_bitwise():
    probs = _small_batch(6, seed=5)
    api = _api()
    params = api.Params(flux=0, cfl=0.4)
    _same(_batched(probs, params, 8, dtype=torch.float32), _loop(probs, params, 8, dtype=torch.float32))


def test_tiles_and_orders_do_not_change_results():
    probs = _small_batch(8, seed=11)
    api = _api()
    ref = None
    for tile in range(len(api.tile_shapes())):
        for order in (0, 1, 2):
            out = _batched(probs, api.Params(flux=1, cfl=0.4, tile=tile), 6, order=order)
            if ref is None:
                ref = out
            else:
                _same(out, ref)


def test_batch_parity_with_oracle():
    probs = _small_batch(6, seed=23)
    api = _api()
    out = _batched(probs, api.Params(flux=1, cfl=0.4), 10)
    for p, (W, A, t, fs, dth) in zip(probs, out):
        Wo, ao, to, dto, fso = O.run(p.W, p.alpha, O.make_grid(p.nx, p.ny, p.dx, p.dy, p.bc_x, p.bc_y),
                                     O.make_params(flux=1, cfl=0.4), 10)
        assert fs == -1 and fso == -1
        err = max(np.abs(W[c] - Wo[c]).sum() / np.abs(Wo[c]).sum() for c in range(4))
        assert err <= 1e-12, (p.nx, p.ny, err)
        assert np.abs(A - ao).sum() / np.abs(ao).sum() <= 1e-12
        np.testing.assert_allclose(dth, dto, rtol=1e-12)


def test_failing_grid_is_isolated():
    probs = _small_batch(5, seed=31)
    bad = probs[2]
    bad.W = bad.W.copy()
    bad.W[3, 0, 0] = -1.0  # negative energy: non-physical input
    api = _api()
    params = api.Params(flux=0, cfl=0.4)
    out = _batched(probs, params, 4)
    ref = _loop(probs, params, 4)
    assert out[2][3] == 0 and ref[2][3] == 0
    for g in (0, 1, 3, 4):
        assert out[g][3] == -1
        assert np.array_equal(out[g][0], ref[g][0])


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_full_ragged_batch_equals_loop(dtype):
    """The 256-grid configuration (sizes log-uniform in [32, 512]), LF, 100 steps.  One Riemann
    grid (60 x 170) meets a non-physical state after 22 steps in FP64 (the CPU oracle fails at the
    same step: the scheme has no positivity limiter); the batch must reproduce the per-grid loop
    bit for bit, failure steps included, and keep every other grid running."""
    probs = WL.batch(256, seed=256, flux=WL.FLUX_LF, cfl=0.4, nsteps=100)
    api = _api()
    params = api.Params(flux=0, cfl=0.4)
    out = _batched(probs, params, 100, dtype=dtype)
    ref = _loop(probs, params, 100, dtype=dtype)
    _same(out, ref)
    failed = [g for g, o in enumerate(out) if o[3] != -1]
    assert len(failed) <= 2, failed
    if dtype == torch.float64:
        assert failed == [161] and out[161][3] == 22


def test_failing_ragged_grid_matches_oracle_up_to_its_failure():
    """Grid 161 of the 256-grid workload: the oracle fails after 22 steps (pinned on the CPU); the
    GPU run equals the oracle through step 21, every cell, and fails at the same step, alone and
    inside the batch."""
    probs = WL.batch(256, seed=256, flux=WL.FLUX_LF, cfl=0.4, nsteps=100)
    p = probs[161]
    g = O.make_grid(p.nx, p.ny, p.dx, p.dy, p.bc_x, p.bc_y)
    Wo, ao, _, dto, fso = O.run(p.W, p.alpha, g, O.make_params(flux=O.FLUX_LF, cfl=0.4), 21)
    assert fso == -1
    api = _api()
    st = api.Stepper.for_problem(p, api.Params(flux=0, cfl=0.4))
    W = torch.tensor(p.W, device="cuda")
    A = torch.tensor(p.alpha, device="cuda")
    dth = torch.zeros(21, dtype=torch.float64, device="cuda")
    _, fs = st.run(W, A, 21, dt_hist=dth)
    assert fs == -1
    Wg, Ag = W.cpu().numpy(), A.cpu().numpy()
    for c in range(4):
        assert np.abs(Wg[c] - Wo[c]).sum() / np.abs(Wo[c]).sum() <= 1e-12
        assert np.abs(Wg[c] - Wo[c]).max() <= 1e-11 * np.abs(Wo[c]).max()
    assert np.abs(Ag - ao).sum() / np.abs(ao).sum() <= 1e-12
    np.testing.assert_allclose(dth.cpu().numpy(), dto, rtol=1e-12)
    _, fs = st.run(W, A, 79)
    assert fs == 1  # the 22nd step fails
    out = _batched([p, probs[160]], api.Params(flux=0, cfl=0.4), 100)
    assert out[0][3] == 22 and out[1][3] == -1


def test_tuned_stepper_matches_default_tile(tmp_path, monkeypatch):
    """Stepper.tuned picks a tile shape by timing the problem itself (cached); results are bitwise
    those of the default tile."""
    monkeypatch.setenv("DFW_TUNE_CACHE", str(tmp_path / "tune.json"))
    api = _api()
    pr = WL.riemann4(96, 80, seed=9)
    params = api.Params(flux=api.FLUX_GKS, cfl=0.4)
    st = api.Stepper.tuned(pr, params)
    assert 0 <= st.params.tile < len(api.tile_shapes())
    ref = api.Stepper.for_problem(pr, params)
    outs = []
    for s in (st, ref):
        W = torch.tensor(pr.W, device="cuda")
        A = torch.tensor(pr.alpha, device="cuda")
        s.run(W, A, 6)
        outs.append((W.cpu().numpy(), A.cpu().numpy()))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    assert (tmp_path / "tune.json").exists()
