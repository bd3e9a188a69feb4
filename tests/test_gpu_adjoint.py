"""Reverse mode (hand-written adjoint with step checkpointing) against the oracle and against
finite differences.

* Whole gradient, element by element, on tiny grids: the oracle's forward-mode derivative (dual
  numbers through its plain FP64 step) along every unit direction gives each entry of
  dJ/d(W^0, alpha^0) for J = <gW, W^N> + <gA, alpha^N>.  Cases: smooth data, a DF field that puts
  part of the grid on the DF branch of eq. (42), transmissive boundaries, LF and GKS; and on grids
  narrower than the stencils (1x9 and 9x1 transmissive strips, a periodic 2x3 grid).
* Dot-product test on larger grids: <grad J, v> against the oracle's directional derivative,
  also on a grid that spans several adjoint tiles in both directions (seams and ragged tails).
* Central differences (eps = 1e-6) of the HIP forward on the 64x64 instance of the adjoint
  workload (density wave plus Gaussian bumps, LF, CFL 0.5, 100 steps, loss = L2 misfit of the
  final density): 8 random unit directions, 8 coordinate directions and the gradient direction;
  and at the workload's full size (1024x1024, the benchmark's configuration): 3 random, 2
  coordinate and the gradient direction.
* Test data keep every kink argument away from zero (|p_l - p_r|, the LF speed max): at an exact
  kink the subgradient each side takes is decided by rounding.
* Rollout (torch.autograd.Function), bitwise determinism, independence of the checkpoint
  interval.
The time step is fixed in every case (dt_fixed), so the oracle and the HIP path take the same dt
without either reading the other's."""
import numpy as np
import pytest

import oracle as O
from paper_2402_10914_amd import workloads as WL

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _api():
    from paper_2402_10914_amd import api
    return api


def _dt_of(pr, cfl):
    smax, ok = O.max_speed(pr.W, O.make_grid(pr.nx, pr.ny, pr.dx, pr.dy, pr.bc_x, pr.bc_y), O.make_params())
    assert ok
    return cfl / smax


def _gpu_grad(pr, flux, dt, nsteps, every, gW, gA):
    api = _api()
    st = api.Stepper.for_problem(pr, api.Params(flux=flux, dt_fixed=dt))
    adj = api.Adjoint(st, nsteps, every)
    W = torch.tensor(pr.W, device="cuda")
    A = torch.tensor(pr.alpha, device="cuda")
    _, fs = adj.forward(W, A)
    assert fs == -1
    gW0, gA0 = adj.backward(torch.tensor(gW, device="cuda"), torch.tensor(gA, device="cuda"))
    return gW0.cpu().numpy(), gA0.cpu().numpy(), W.cpu().numpy(), A.cpu().numpy()


def _oracle_directional(pr, flux, dt, nsteps, vW, vA, gW, gA):
    g = O.make_grid(pr.nx, pr.ny, pr.dx, pr.dy, pr.bc_x, pr.bc_y)
    _, _, dW, dA = O.run_tangent(pr.W, pr.alpha, vW, vA, g, O.make_params(flux=flux, dt_fixed=dt), [dt] * nsteps)
    return float((gW * dW).sum() + (gA * dA).sum())


def _oracle_full_grad(pr, flux, dt, nsteps, gW, gA):
    N = pr.nx * pr.ny
    out = np.zeros(5 * N)
    for k in range(5 * N):
        vW = np.zeros((4, pr.ny, pr.nx))
        vA = np.zeros((pr.ny, pr.nx))
        if k < 4 * N:
            vW.reshape(-1)[k] = 1.0
        else:
            vA.reshape(-1)[k - 4 * N] = 1.0
        out[k] = _oracle_directional(pr, flux, dt, nsteps, vW, vA, gW, gA)
    return out[: 4 * N].reshape(4, pr.ny, pr.nx), out[4 * N:].reshape(pr.ny, pr.nx)


def _seeds(pr, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((4, pr.ny, pr.nx)), rng.standard_normal((pr.ny, pr.nx))


def _tiny(case):
    if case == "smooth":
        pr = WL.density_wave(7, 6)
        rng = np.random.default_rng(70)
        pr.W = pr.W * (1.0 + 0.01 * rng.standard_normal(pr.W.shape))
    elif case == "df":
        # periodic: a block of higher density and pressure over random cell states.  Pressure and
        # velocity vary from cell to cell, so no kink argument (|p_l - p_r| of the DF and of the
        # GKS collision time, the LF speed max) sits at zero, where the subgradient would be
        # decided by rounding.
        pr = WL.density_wave(7, 6)
        rng = np.random.default_rng(71)
        rho = 1.0 + 0.2 * rng.random((6, 7))
        p = 1.0 + 0.3 * rng.random((6, 7))
        rho[2:5, 3:6] *= 3.0
        p[2:5, 3:6] *= 2.0
        u = 1.0 + 0.2 * rng.standard_normal((6, 7))
        v = 0.5 + 0.2 * rng.standard_normal((6, 7))
        pr.W = np.stack([rho, rho * u, rho * v, p / (WL.GAMMA - 1.0) + 0.5 * rho * (u * u + v * v)])
        a = rng.uniform(0.6, 1.0, (6, 7))
        a[1:5, 1:4] = rng.uniform(0.1, 0.45, (4, 3))  # DF branch where the 3-cell max is below 0.5
        pr.alpha = a
    elif case == "transmissive":
        pr = WL.riemann4(7, 6, seed=8)
        rng = np.random.default_rng(72)
        pr.alpha = rng.uniform(0.3, 1.0, (6, 7))
    else:
        raise ValueError(case)
    return pr


def _rel_l1(a, b):
    scale = np.abs(b).sum()
    if scale == 0.0:  # e.g. no derivative to alpha^0 when no cell is on the DF branch
        return float(np.abs(a).max())
    return float(np.abs(a - b).sum() / scale)


@pytest.mark.parametrize("flux", [WL.FLUX_LF, WL.FLUX_GKS])
@pytest.mark.parametrize("case", ["smooth", "df", "transmissive"])
def test_whole_gradient_matches_oracle_forward_mode(case, flux):
    pr = _tiny(case)
    assert (pr.bc_x == WL.BC_TRANSMISSIVE) == (case == "transmissive")
    nsteps, every = 3, 2
    dt = _dt_of(pr, 0.4)
    gW, gA = _seeds(pr, 5)
    gW0, gA0, _, _ = _gpu_grad(pr, flux, dt, nsteps, every, gW, gA)
    oW, oA = _oracle_full_grad(pr, flux, dt, nsteps, gW, gA)
    assert _rel_l1(gW0, oW) <= 1e-10
    assert _rel_l1(gA0, oA) <= 1e-10
    if case == "df":  # the DF branch carries derivative to alpha^0 through the blend
        assert np.abs(oA).max() > 1e-3


def _degenerate(case):
    rng = np.random.default_rng(73)
    if case == "strip_x":  # one cell wide along x, transmissive
        pr = WL.riemann4(1, 9, seed=8)
    elif case == "strip_y":  # one cell high along y, transmissive
        pr = WL.riemann4(9, 1, seed=8)
    elif case == "periodic_2x3":  # smaller than every stencil in both directions, periodic
        pr = WL.density_wave(2, 3)
        pr.W = pr.W * (1.0 + 0.01 * rng.standard_normal(pr.W.shape))
    else:
        raise ValueError(case)
    pr.alpha = rng.uniform(0.1, 1.0, (pr.ny, pr.nx))  # some cells on the DF branch
    return pr


@pytest.mark.parametrize("flux", [WL.FLUX_LF, WL.FLUX_GKS])
@pytest.mark.parametrize("case", ["strip_x", "strip_y", "periodic_2x3"])
def test_whole_gradient_on_degenerate_grids(case, flux):
    # grids narrower than the stencils: ghost cells fold back through the boundary map many times,
    # in the tile staging, the seed staging and the gather
    pr = _degenerate(case)
    nsteps, every = 3, 2
    dt = _dt_of(pr, 0.4)
    gW, gA = _seeds(pr, 7)
    gW0, gA0, _, _ = _gpu_grad(pr, flux, dt, nsteps, every, gW, gA)
    oW, oA = _oracle_full_grad(pr, flux, dt, nsteps, gW, gA)
    assert _rel_l1(gW0, oW) <= 1e-10, (case, _rel_l1(gW0, oW))
    assert _rel_l1(gA0, oA) <= 1e-10, (case, _rel_l1(gA0, oA))
    if case == "periodic_2x3":  # the DF branch carries derivative to alpha^0 (the strips' data are
        assert np.abs(oA).max() > 1e-3  # constant along the DF-branch stencils)


@pytest.mark.parametrize("flux", [WL.FLUX_LF, WL.FLUX_GKS])
def test_dot_product_against_oracle_directional_derivative(flux):
    pr = WL.riemann4(40, 33, seed=11)
    nsteps, every = 9, 4
    dt = _dt_of(pr, 0.4)
    gW, gA = _seeds(pr, 6)
    gW0, gA0, _, A = _gpu_grad(pr, flux, dt, nsteps, every, gW, gA)
    rng = np.random.default_rng(12)
    for _ in range(3):
        vW = rng.standard_normal(pr.W.shape)
        vA = rng.standard_normal(pr.alpha.shape)
        ref = _oracle_directional(pr, flux, dt, nsteps, vW, vA, gW, gA)
        got = float((gW0 * vW).sum() + (gA0 * vA).sum())
        assert abs(got - ref) <= 1e-10 * abs(ref), (got, ref)


def _random_states(nx, ny, seed):
    """Periodic grid of random cell states (no two neighbouring pressures equal, so no kink argument
    sits at zero), a denser block, and alpha partly below the DF threshold."""
    pr = WL.density_wave(nx, ny)
    rng = np.random.default_rng(seed)
    rho = 1.0 + 0.2 * rng.random((ny, nx))
    p = 1.0 + 0.3 * rng.random((ny, nx))
    rho[ny // 3: ny // 2, nx // 4: nx // 2] *= 3.0
    p[ny // 3: ny // 2, nx // 4: nx // 2] *= 2.0
    u = 1.0 + 0.2 * rng.standard_normal((ny, nx))
    v = 0.5 + 0.2 * rng.standard_normal((ny, nx))
    pr.W = np.stack([rho, rho * u, rho * v, p / (WL.GAMMA - 1.0) + 0.5 * rho * (u * u + v * v)])
    pr.alpha = rng.uniform(0.1, 1.0, (ny, nx))
    return pr


@pytest.mark.parametrize("flux", [WL.FLUX_LF, WL.FLUX_GKS])
@pytest.mark.parametrize("case", ["transmissive", "periodic_df"])
def test_dot_product_across_adjoint_tile_seams(case, flux):
    # 126 x 67: the x-interfaces span two 60-row adjoint tiles (the second ragged, 7 rows) and the
    # y-interfaces three (the last 6 columns), so segment rows on both sides of every seam and the
    # tails are reversed by different workgroups and summed by the gather
    pr = WL.riemann4(126, 67, seed=13) if case == "transmissive" else _random_states(126, 67, 14)
    nsteps, every = 4, 3
    dt = _dt_of(pr, 0.4)
    gW, gA = _seeds(pr, 15)
    gW0, gA0, _, _ = _gpu_grad(pr, flux, dt, nsteps, every, gW, gA)
    rng = np.random.default_rng(16)
    for _ in range(3):
        vW = rng.standard_normal(pr.W.shape)
        vA = rng.standard_normal(pr.alpha.shape)
        ref = _oracle_directional(pr, flux, dt, nsteps, vW, vA, gW, gA)
        got = float((gW0 * vW).sum() + (gA0 * vA).sum())
        assert abs(got - ref) <= 1e-10 * abs(ref), (case, got, ref)


def _bumps_loss_setup(n=64, nsteps=100):
    pr = WL.bumps(n, seed=1024)
    dt = _dt_of(pr, 0.5)
    target = WL.bumps_target(n, nsteps * dt, seed=1025)
    return pr, dt, target


def _loss(api, st, W0, A0, nsteps, target_t, area):
    W = W0.clone()
    A = A0.clone()
    _, fs = st.run(W, A, nsteps)
    assert fs == -1
    return 0.5 * area * float(((W[0] - target_t) ** 2).sum())


def _central_differences(n, n_random, n_coord, seed):
    """The adjoint workload's loss on an n x n instance (density wave plus Gaussian bumps, LF, CFL 0.5,
    100 steps, checkpoints every 10): the gradient against central differences (eps = 1e-6) of the HIP
    forward along n_random random unit directions, n_coord coordinate directions spread over the
    large entries, and the gradient direction."""
    nsteps, eps = 100, 1e-6
    pr, dt, target = _bumps_loss_setup(n, nsteps)
    api = _api()
    st = api.Stepper.for_problem(pr, api.Params(flux=api.FLUX_LF, dt_fixed=dt))
    W0 = torch.tensor(pr.W, device="cuda")
    A0 = torch.tensor(pr.alpha, device="cuda")
    tt = torch.tensor(target, device="cuda")
    area = pr.dx * pr.dy
    adj = api.Adjoint(st, nsteps, 10)
    W = W0.clone()
    A = A0.clone()
    adj.forward(W, A)
    gW = torch.zeros_like(W)
    gW[0] = area * (W[0] - tt)
    gW0, _ = adj.backward(gW, None)
    g = gW0.cpu().numpy()
    rng = np.random.default_rng(seed)
    dirs = []
    for _ in range(n_random):
        v = rng.standard_normal(pr.W.shape)
        dirs.append(v / np.linalg.norm(v))
    flat = np.argsort(np.abs(g).ravel())[::-1]
    for k in flat[:: max(1, len(flat) // 64)][:n_coord]:  # coordinate directions spread over the large entries
        v = np.zeros(pr.W.size)
        v[k] = 1.0
        dirs.append(v.reshape(pr.W.shape))
    gnorm = float(np.linalg.norm(g))
    dirs.append(g / gnorm)
    # relative to the directional derivative; for directions nearly orthogonal to the gradient the
    # rounding floor of the differences (about eps_mach J / eps) dominates, hence the floor at 1%
    # of |grad J| (a unit direction's derivative is at most |grad J|)
    worst = 0.0
    for v in dirs:
        vt = torch.tensor(v, device="cuda")
        jp = _loss(api, st, W0 + eps * vt, A0, nsteps, tt, area)
        jm = _loss(api, st, W0 - eps * vt, A0, nsteps, tt, area)
        fd = (jp - jm) / (2 * eps)
        ad = float((g * v).sum())
        scale = max(abs(ad), 1e-2 * gnorm)
        assert abs(fd - ad) <= 1e-6 * scale, (n, fd, ad, gnorm)
        worst = max(worst, abs(fd - ad) / scale)
    print(f"bumps{n} central differences: {len(dirs)} directions, worst relative difference {worst:.2e}", flush=True)


def test_central_differences_on_bumps64():
    _central_differences(64, 8, 8, 64)


def test_central_differences_at_full_size_1024():
    # the adjoint benchmark's grid, steps, checkpoint interval and launch configuration; the pressure
    # of this workload is uniform, so the GKS collision time's |p_l - p_r| sits at its kink, where
    # differences and the subgradient part ways: LF only
    _central_differences(1024, 3, 2, 1024)


def test_rollout_autograd_function_and_gradcheck():
    api = _api()
    pr = WL.riemann4(10, 8, seed=21)
    dt = _dt_of(pr, 0.4)
    st = api.Stepper.for_problem(pr, api.Params(flux=api.FLUX_LF, dt_fixed=dt))
    W0 = torch.tensor(pr.W, device="cuda", requires_grad=True)
    A0 = torch.tensor(pr.alpha, device="cuda", requires_grad=True)
    R = torch.randn(4, 8, 10, dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(3))
    WN, AN = api.rollout(W0, A0, st, 4, 3)
    J = (WN * R).sum() + AN.sum()
    J.backward()
    adj = api.Adjoint(st, 4, 3)
    W = W0.detach().clone()
    A = A0.detach().clone()
    adj.forward(W, A)
    assert torch.equal(W, WN.detach()) and torch.equal(A, AN.detach())
    gW0, gA0 = adj.backward(R.clone(), torch.ones_like(A))
    assert torch.equal(W0.grad, gW0) and torch.equal(A0.grad, gA0)
    Wc = W0.detach().clone().requires_grad_(True)
    Ac = A0.detach().clone().requires_grad_(True)
    assert torch.autograd.gradcheck(lambda w, a: api.rollout(w, a, st, 2, 1), (Wc, Ac), eps=1e-6, atol=1e-7,
                                    rtol=1e-5, fast_mode=True)


def test_deterministic_and_independent_of_checkpoint_interval():
    pr = WL.riemann4(37, 29, seed=13)
    dt = _dt_of(pr, 0.4)
    gW, gA = _seeds(pr, 9)
    ref = _gpu_grad(pr, WL.FLUX_GKS, dt, 7, 3, gW, gA)
    for every in (3, 1, 7, 100):
        out = _gpu_grad(pr, WL.FLUX_GKS, dt, 7, every, gW, gA)
        assert np.array_equal(out[0], ref[0]) and np.array_equal(out[1], ref[1]), every


@pytest.mark.parametrize("flux", [WL.FLUX_LF, WL.FLUX_GKS])
@pytest.mark.parametrize("n", [64, 1024])
def test_full_record_equals_checkpointed_gradient(n, flux):
    """ckpt_every = 1 (each step recorded whole by the forward run, nothing recomputed) against
    checkpoints every ten steps on the n x n instance of the adjoint workload, 100 steps (n = 1024:
    its full size, 9.2 GB of records): the same final state and the same gradient (W and alpha), bit
    for bit."""
    nsteps = 100
    pr, dt, target = _bumps_loss_setup(n, nsteps)
    api = _api()
    st = api.Stepper.for_problem(pr, api.Params(flux=flux, dt_fixed=dt))
    area = pr.dx * pr.dy
    out = []
    for every in (10, 1):
        adj = api.Adjoint(st, nsteps, every)
        W = torch.tensor(pr.W, device="cuda")
        A = torch.tensor(pr.alpha, device="cuda")
        _, fs = adj.forward(W, A)
        assert fs == -1
        gW = torch.zeros_like(W)
        gW[0] = area * (W[0] - torch.tensor(target, device="cuda"))
        gW0, gA0 = adj.backward(gW, torch.ones_like(A))
        out.append([x.cpu().numpy() for x in (W, A, gW0, gA0)])
    for a, b in zip(*out):
        assert np.array_equal(a, b)
    assert np.abs(out[0][2]).max() > 0


@pytest.mark.parametrize("every", [10, 1])
def test_zero_steps_is_identity(every):
    pr = WL.riemann4(9, 11, seed=2)
    gW, gA = _seeds(pr, 1)
    gW0, gA0, _, _ = _gpu_grad(pr, WL.FLUX_LF, 1e-3, 0, every, gW, gA)
    assert np.array_equal(gW0, gW) and np.array_equal(gA0, gA)
