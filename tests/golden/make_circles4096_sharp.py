"""Writes circles4096_sharp_gks.json: the oracle's run of the 4096x4096 circles workload with sharp,
point-sampled circular regions (edge_cells = 0; periodic [0,2]^2, seed 10914, WENO-AO + DF, S2O4,
GKS, CFL 0.4): the step at which it meets a non-physical cell average, the time reached, the time
steps taken and the non-physical cells of the state it stops at.

    OMP_NUM_THREADS=8 python tests/golden/make_circles4096_sharp.py     (about 6 minutes on 8 cores)

Calls only the oracle and the seeded input generator."""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
from paper_2402_10914_amd import workloads as WL  # noqa: E402

N, SEED, CFL, STEPS = 4096, 10914, 0.4, 4
OUT = os.path.join(HERE, "circles4096_sharp_gks.json")


def nonphysical(W, gamma=1.4):
    p = (gamma - 1.0) * (W[3] - 0.5 * (W[1] ** 2 + W[2] ** 2) / W[0])
    return ~(np.isfinite(W).all(axis=0) & (W[0] > 0) & (p > 0))


def main():
    pr = WL.circles(N, seed=SEED, cfl=CFL, edge_cells=0)
    g = O.make_grid(N, N, pr.dx, pr.dy, pr.bc_x, pr.bc_y)
    W, _, t, dth, fs = O.run(pr.W, pr.alpha, g, O.make_params(flux=O.FLUX_GKS, cfl=CFL), STEPS)
    bad = nonphysical(W)
    jj, ii = np.nonzero(bad)
    with open(OUT, "w") as f:
        json.dump({"workload": "4096x4096 circles, sharp point-sampled edges, GKS, WENO-AO+DF, S2O4, CFL 0.4",
                   "steps_requested": STEPS, "fail_step": int(fs), "t": float(t), "dt_hist": [float(x) for x in dth],
                   "nonphysical_cells": [[int(j), int(i)] for j, i in zip(jj, ii)]}, f, indent=1)
    print("fail step", fs, "t", t, "cells", len(jj))


if __name__ == "__main__":
    main()
