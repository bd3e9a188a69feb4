"""Writes circles4096_<flux>_50.npz: the oracle's state after 50 steps of the 4096x4096 circles
workload (periodic [0,2]^2, seed 10914, 32 circular regions with two-cell tanh edges; WENO-AO + DF,
S2O4, CFL 0.4) for the GKS or the LF flux, sampled at 4096 seeded cells, at the 4096 cells of the
final state with the largest pressure jump to the east neighbour (the fronts, where the hybrid
switch and the DF act), and along the two centre lines; with the dt history, the final time and
the per-component sums.

    OMP_NUM_THREADS=6 python tests/golden/make_circles4096.py gks   (about 2.5 hours on 6 cores)
    OMP_NUM_THREADS=6 python tests/golden/make_circles4096.py lf    (about 1.2 hours)

Calls only the oracle and the seeded input generator."""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
from paper_2402_10914_amd import workloads as WL  # noqa: E402

N, STEPS, SEED, CFL = 4096, 50, 10914, 0.4


def sample_cells(n, k=4096, seed=4096):
    rng = np.random.default_rng(seed)
    return rng.integers(0, n, k), rng.integers(0, n, k)


def front_cells(W, k=4096, gamma=1.4):
    p = (gamma - 1) * (W[3] - 0.5 * (W[1] ** 2 + W[2] ** 2) / W[0])
    jump = np.abs(np.roll(p, -1, axis=1) - p) / p
    flat = np.argpartition(jump.ravel(), -k)[-k:]
    flat = np.sort(flat)
    return flat // W.shape[-1], flat % W.shape[-1]


def path(name):
    return os.path.join(HERE, f"circles4096_{name}_50.npz")


def main(name):
    flux = {"gks": O.FLUX_GKS, "lf": O.FLUX_LF}[name]
    pr = WL.circles(N, seed=SEED, cfl=CFL, nsteps=STEPS)
    g = O.make_grid(N, N, pr.dx, pr.dy, pr.bc_x, pr.bc_y)
    p = O.make_params(flux=flux, cfl=CFL)
    t0 = time.time()
    W, a, t, dth, fs = O.run(pr.W, pr.alpha, g, p, STEPS)
    assert fs == -1
    jj, ii = sample_cells(N)
    fj, fi = front_cells(W)
    np.savez_compressed(path(name), jj=jj, ii=ii, W_s=W[:, jj, ii], a_s=a[jj, ii], fj=fj, fi=fi,
                        W_f=W[:, fj, fi], a_f=a[fj, fi], W_row=W[:, N // 2, :], W_col=W[:, :, N // 2],
                        a_row=a[N // 2, :], a_col=a[:, N // 2], dt_hist=dth, t=t, sums=W.sum(axis=(1, 2)),
                        abs_sums=np.abs(W).sum(axis=(1, 2)), alpha_min=a.min())
    print(name, "t", t, "alpha min", a.min(), f"{time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "gks")
