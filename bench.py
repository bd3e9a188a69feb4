#!/usr/bin/env python3
"""Benchmark of the S2O4 DF-hybrid step (Zhang, Ji & Xu, arXiv:2402.10914) on one MI355X.

Default workload: 2-D Euler, FP64, 4096 x 4096 cells on periodic [0,2]^2: a density-wave background
with 32 seeded circular regions (seed 10914; density ratios up to 10, pressure ratios up to 1e3; each
region's edge smoothed over two cells by a tanh profile, since the scheme has no positivity limiter
and fails in the first step on point-sampled sharp edges), gas-kinetic flux, WENO-AO + DF, S2O4,
CFL 0.4, the first 50 steps of the run.  One "step" is one S2O4 time step of the whole grid (all
parts of the path: CFL reduction, ghost fill, DF, reconstruction, fluxes with time derivatives,
two-stage update).  The timed region runs exactly --steps steps from the initial condition after
--warmup untimed steps; inputs are resident in HBM before timing starts.  The interface tile shape
is the autotuner's pick for this grid (--tile overrides it).  --workload circles4096_lf (LF flux),
circles4096_gks_f32 / circles4096_lf_f32 (FP32) and riemann512_gks / riemann512_lf (512 x 512
four-quadrant Riemann data, transmissive) select the other configurations.

Prints one JSON line: cell-updates/s, per-kernel roofline of the dominant kernel (FP64 vector ALU
bound: its algorithmic flops per launch over its mean launch time, measured with HIP events on the
launch stream) and the CPU oracle timed on a bounded sample on this host.

Also reported: the batched form against the per-grid loop ("batched"), the cost of the gradient of
a 100-step rollout against the rollout itself ("adjoint"), and the circles workload as configured,
with sharp point-sampled edges, on the LF flux, which runs it ("sharp_edges_lf").

Other modes:  --mode copy      plain device copy of known size (calibrates rocprofv3 FETCH/WRITE_SIZE).
              --mode adjoint   the gradient measurement alone.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_VALU = 78.6   # TFLOP/s, MI355X FP64 vector
PEAK_FP32_VALU = 157.3  # TFLOP/s, MI355X FP32 vector
PEAK_HBM = 8000.0       # GB/s
BYTES_PER_CELL_UPDATE = {8: 216, 4: 108}  # algorithmic HBM bytes of one S2O4 step per cell


def _code_only(src: str) -> str:
    """Source text without comments and whitespace (so that edits of comments keep the hash)."""
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    src = re.sub(r"//[^\n]*", "", src)
    return re.sub(r"\s+", "", src)


def kernel_source_hash(read=None):
    """Hash of the code of the forward kernels (dfw_math.hpp, dfw_step.hip)."""
    h = hashlib.sha256()
    for f in ("dfw_math.hpp", "dfw_step.hip"):
        path = os.path.join(ROOT, "paper_2402_10914_amd", "csrc", f)
        if read:
            text = read(f)
        else:
            with open(path) as fh:
                text = fh.read()
        h.update(_code_only(text).encode())
    return h.hexdigest()[:16]


def load_traffic(name):
    """HBM bytes per launch from committed rocprofv3 counter runs, if taken on the current kernels."""
    p = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(p):
        return None
    with open(p) as f:
        d = json.load(f)
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    return d.get("bytes_per_launch")


def workload(name):
    from paper_2402_10914_amd import workloads as WL
    if name == "riemann512_gks":
        return WL.riemann4(512, seed=2402, flux=WL.FLUX_GKS, cfl=0.4, nsteps=200), "f64"
    if name == "riemann512_lf":
        return WL.riemann4(512, seed=2402, flux=WL.FLUX_LF, cfl=0.4, nsteps=200), "f64"
    if name in ("circles4096_gks", "circles4096_lf", "circles4096_gks_f32", "circles4096_lf_f32"):
        flux = WL.FLUX_GKS if "gks" in name else WL.FLUX_LF
        return WL.circles(4096, seed=10914, flux=flux, cfl=0.4, nsteps=50), ("f32" if name.endswith("f32") else "f64")
    raise SystemExit(f"unknown workload {name}")


def workload_text(prob, tl, ts):
    flux = "GKS" if prob.flux else "LF"
    scheme = f"{'SSP-RK3' if ts else 'S2O4'}{', time limiter' if tl else ''}"
    if prob.name == "riemann4":
        return f"{prob.nx}x{prob.ny} four-quadrant Riemann, {flux}, WENO-AO+DF, {scheme}, CFL 0.4, transmissive"
    return (f"{prob.nx}x{prob.ny} periodic density wave + 32 circles (rho ratio <= 10, p ratio <= 1e3, "
            f"edges tanh-smoothed over 2 cells), {flux}, WENO-AO+DF, {scheme}, CFL 0.4, first 50 steps")


def cpu_baseline(prob, steps, cells, time_limiter=0, time_scheme=0):
    """The oracle as it stands on this host: `steps` steps of the central cells x cells part of the
    workload's initial state (the whole grid when it is smaller), same boundary types."""
    import numpy as np

    import oracle as O
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    nx, ny = min(cells, prob.nx), min(cells, prob.ny)
    i0, j0 = (prob.nx - nx) // 2, (prob.ny - ny) // 2
    W = np.ascontiguousarray(prob.W[:, j0:j0 + ny, i0:i0 + nx])
    A = np.ascontiguousarray(prob.alpha[j0:j0 + ny, i0:i0 + nx])
    g = O.make_grid(nx, ny, prob.dx, prob.dy, prob.bc_x, prob.bc_y)
    p = O.make_params(flux=prob.flux, cfl=prob.cfl, time_limiter=time_limiter, time_scheme=time_scheme)
    t0 = time.perf_counter()
    O.run(W, A, g, p, steps)
    el = time.perf_counter() - t0
    part = "the whole grid" if (nx, ny) == (prob.nx, prob.ny) else f"the central {nx}x{ny} cells of the {prob.nx}x{prob.ny} grid"
    return {"value": nx * ny * steps / el, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{steps} {'SSP-RK3' if time_scheme else 'S2O4'} step(s) of {part} from the same initial state, "
                      f"same flux and boundary types ({el:.1f} s, OpenMP over rows)"}


def batch_compare(nsteps=100, tune=True, dtype_name="f64"):
    """Ragged batch of 256 grids (LF, FP64 or FP32): one captured-graph replay against the per-grid
    loop, both with the tile and order the autotuner picks for the batch."""
    import torch
    from paper_2402_10914_amd import api, autotune
    from paper_2402_10914_amd import workloads as WL
    dtype = torch.float64 if dtype_name == "f64" else torch.float32
    probs = WL.batch(256, seed=256, flux=WL.FLUX_LF, cfl=0.4, nsteps=nsteps)
    grids = [(p.nx, p.ny, p.dx, p.dy, p.bc_x, p.bc_y) for p in probs]
    params = api.Params(flux=api.FLUX_LF, cfl=0.4)
    tile, order = 0, 0
    if tune:
        tile, order, _ = autotune.tune_batch(grids, [p.W for p in probs], [p.alpha for p in probs], params, dtype,
                                             steps=5)
        params = api.Params(flux=api.FLUX_LF, cfl=0.4, tile=tile)
    cells = sum(p.nx * p.ny for p in probs)
    b = api.Batch(grids, params, dtype, order)
    W0, A0 = b.pack([p.W for p in probs], [p.alpha for p in probs])
    W, A = W0.clone(), A0.clone()
    b.run(W, A, nsteps, use_graph=True)  # capture
    W.copy_(W0)
    A.copy_(A0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, fs = b.run(W, A, nsteps, use_graph=True)
    torch.cuda.synchronize()
    t_graph = time.perf_counter() - t0
    steppers = [api.Stepper.for_problem(p, params, dtype) for p in probs]
    Ws = [torch.tensor(p.W, dtype=dtype, device="cuda") for p in probs]
    As = [torch.tensor(p.alpha, dtype=dtype, device="cuda") for p in probs]
    for st, w, a in zip(steppers, Ws, As):  # warm
        st.run(w.clone(), a.clone(), 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fl = [st.run(w, a, nsteps)[1] for st, w, a in zip(steppers, Ws, As)]
    torch.cuda.synchronize()
    t_loop = time.perf_counter() - t0
    views = b.unpack(W, A)
    same = all(bool(torch.equal(torch.nan_to_num(v[0]), torch.nan_to_num(w))) and bool(torch.equal(torch.nan_to_num(v[1]), torch.nan_to_num(a))) for v, w, a in zip(views, Ws, As))
    # grids that meet a non-physical state stop there (in both forms): count executed updates only
    done = sum(p.nx * p.ny * (nsteps if f == -1 else f) for p, f in zip(probs, fs))
    return {"grids": len(probs), "cells": cells, "steps": nsteps, "dtype": dtype_name, "flux": "lf",
            "executed_cell_updates": done,
            "graph_cell_updates_per_s": done / t_graph, "loop_cell_updates_per_s": done / t_loop,
            "speedup": t_loop / t_graph, "bitwise_equal": same and list(fs) == fl, "tile": tile, "order": order,
            "graph_ms": t_graph * 1e3, "loop_ms": t_loop * 1e3, "failed_grids": sum(1 for f in fs if f != -1)}


def adjoint_compare(n=1024, nsteps=100, every=10, flux="lf", tape=True):
    """Adjoint workload (FP64, n x n periodic density wave plus 16 Gaussian bumps, LF (or GKS),
    CFL 0.5, nsteps steps, checkpoint every `every` steps, loss = L2 misfit of the final density to a
    seeded target): time of the gradient (segment recomputation and reverse sweep) over the time of
    the plain forward rollout.  With `tape`, also the same with a checkpoint at every step (the
    forward run keeps each step's whole record, the gradient recomputes nothing), and whether its
    gradient equals the first bitwise."""
    import torch
    from paper_2402_10914_amd import api
    from paper_2402_10914_amd import workloads as WL
    prob = WL.bumps(n, seed=1024, cfl=0.5, nsteps=nsteps)
    fl = {"lf": api.FLUX_LF, "gks": api.FLUX_GKS}[flux]
    st = api.Stepper.for_problem(prob, api.Params(flux=fl, cfl=0.5))
    W0 = torch.tensor(prob.W, device="cuda")
    A0 = torch.tensor(prob.alpha, device="cuda")
    adj = api.Adjoint(st, nsteps, every)

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0, r

    W, A = W0.clone(), A0.clone()
    st.run(W, A, 2)  # warm
    W, A = W0.clone(), A0.clone()
    t_fwd, (t_sim, fs) = timed(lambda: st.run(W, A, nsteps))
    W, A = W0.clone(), A0.clone()
    t_fwd_ckpt, _ = timed(lambda: adj.forward(W, A))
    target = torch.tensor(WL.bumps_target(n, t_sim, seed=1025), device="cuda")
    area = prob.dx * prob.dy
    gW = torch.zeros_like(W)
    gW[0] = area * (W[0] - target)
    loss = 0.5 * area * float(((W[0] - target) ** 2).sum())
    adj.backward(gW, None)  # warm
    t_bwd, (gW0, _) = timed(lambda: adj.backward(gW, None))
    with api.KernelProfile() as kp:
        adj.backward(gW, None)
    prof = kp.result()
    kernels = {k: {"avg_us": round(1e3 * ms / c, 2), "launches": c, "total_ms": round(ms, 3)}
               for k, (ms, c) in prof.items() if c}
    recompute_ms = sum(prof[k][0] for k in ("faces1", "update1", "faces2", "update2"))
    reverse_ms = sum(prof[k][0] for k in ("adj_faces1", "adj_faces2", "adj_gather"))
    ckpt_bytes, ws_bytes = adj.ckpt_bytes, adj.ws_bytes
    full = None
    if tape:
        del adj
        torch.cuda.empty_cache()
        adj1 = api.Adjoint(st, nsteps, 1)
        W, A = W0.clone(), A0.clone()
        t_fwd1, _ = timed(lambda: adj1.forward(W, A))
        adj1.backward(gW, None)  # warm
        t_bwd1, (gW1, _) = timed(lambda: adj1.backward(gW, None))
        full = {"ckpt_every": 1, "forward_with_record_ms": round(t_fwd1 * 1e3, 2),
                "gradient_ms": round(t_bwd1 * 1e3, 2), "ratio_gradient_over_forward": round(t_bwd1 / t_fwd, 3),
                "checkpoint_bytes": adj1.ckpt_bytes, "workspace_bytes": adj1.ws_bytes,
                "gradient_bitwise_equal": bool(torch.equal(gW1, gW0))}
        del adj1
        torch.cuda.empty_cache()
    return {"grid": f"{n}x{n}", "steps": nsteps, "ckpt_every": every, "flux": flux, "dtype": "f64", "full_record": full,
            "forward_ms": round(t_fwd * 1e3, 2), "forward_with_checkpoints_ms": round(t_fwd_ckpt * 1e3, 2),
            "gradient_ms": round(t_bwd * 1e3, 2), "ratio_gradient_over_forward": round(t_bwd / t_fwd, 3),
            "recompute_kernels_ms": round(recompute_ms, 2), "reverse_kernels_ms": round(reverse_ms, 2),
            "loss": loss, "grad_norm": float(gW0.norm()), "fail_step": fs,
            "checkpoint_bytes": ckpt_bytes, "workspace_bytes": ws_bytes, "kernels": kernels}


def sharp_lf_leg(steps=20, warmup=3, tile=-1):
    """The 4096x4096 circles workload as configured, with sharp point-sampled regions, on the LF flux
    (which runs it; GKS meets a non-physical state after 3 steps there, as the oracle does)."""
    import torch
    from paper_2402_10914_amd import api
    from paper_2402_10914_amd import workloads as WL
    prob = WL.circles(4096, seed=10914, flux=WL.FLUX_LF, cfl=0.4, nsteps=50, edge_cells=0)
    params = api.Params(flux=api.FLUX_LF, cfl=0.4, tile=max(tile, 0))
    st = api.Stepper.for_problem(prob, params) if tile >= 0 else api.Stepper.tuned(prob, params)
    W0 = torch.tensor(prob.W, device="cuda")
    A0 = torch.tensor(prob.alpha, device="cuda")
    W, A = W0.clone(), A0.clone()
    st.run(W, A, warmup)
    W.copy_(W0)
    A.copy_(A0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, fail = st.run(W, A, steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    done = steps if fail == -1 else fail
    return {"workload": "4096x4096 periodic density wave + 32 circles with sharp point-sampled edges (rho ratio "
                        "<= 10, p ratio <= 1e3), LF, WENO-AO+DF, S2O4, CFL 0.4", "dtype": "f64",
            "value": prob.nx * prob.ny * done / el, "unit": "cell-updates/s", "steps": steps,
            "ms_per_step": el * 1e3 / steps, "fail_step": fail, "tile": st.params.tile}


def copy_mode(args):
    import torch
    n = 1 << 26  # 64 Mi doubles = 512 MiB each way
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(args.warmup):
        b.copy_(a)
    torch.cuda.synchronize()
    for _ in range(args.steps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"mode": "copy", "bytes_read_per_launch": 8 * n, "bytes_written_per_launch": 8 * n,
                      "launches": args.steps}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="circles4096_gks")
    ap.add_argument("--tile", type=int, default=-1, help="interface tile shape (default: the autotuner's pick)")
    ap.add_argument("--cpu-steps", type=int, default=1)
    ap.add_argument("--cpu-cells", type=int, default=2048,
                    help="the CPU baseline runs the oracle on the central cpu-cells x cpu-cells part of the grid")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-sharp", action="store_true", help="skip the sharp-edged LF run of the circles workload")
    ap.add_argument("--mode", default="step", choices=["step", "copy", "adjoint"])
    ap.add_argument("--time-limiter", action="store_true", help="the non-linear time limiter (the paper's GKS solver)")
    ap.add_argument("--ssprk3", action="store_true", help="SSP-RK3 time steps (the paper's LF solver; LF workloads)")
    ap.add_argument("--adjoint-flux", default="lf", choices=["lf", "gks"], help="flux of --mode adjoint")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures the step on a single MI355X (the library has no multi-GPU path); "
              f"--gpus {args.gpus} / WORLD_SIZE {world} is not supported.", file=sys.stderr)
        sys.exit(2)
    if args.mode == "copy":
        return copy_mode(args)
    if args.mode == "adjoint":
        print(json.dumps({"mode": "adjoint", **adjoint_compare(flux=args.adjoint_flux)}))
        return

    import torch
    from paper_2402_10914_amd import api, flops

    prob, dt_name = workload(args.workload)
    dtype = torch.float64 if dt_name == "f64" else torch.float32
    esize = 8 if dtype == torch.float64 else 4
    tl, ts = int(args.time_limiter), int(args.ssprk3)
    if ts and (prob.flux != api.FLUX_LF or tl):
        raise SystemExit("--ssprk3 runs with the LF flux and without the time limiter")
    params = api.Params(flux=prob.flux, cfl=prob.cfl, time_limiter=tl, time_scheme=ts)
    default_form = not (tl or ts)
    if args.tile >= 0:
        params.tile = args.tile
        st = api.Stepper.for_problem(prob, params, dtype)
    else:
        st = api.Stepper.tuned(prob, params, dtype)
        params = st.params
    W0 = torch.tensor(prob.W, dtype=dtype, device="cuda")
    A0 = torch.tensor(prob.alpha, dtype=dtype, device="cuda")
    W = W0.clone()
    A = A0.clone()
    print(f"# workload {args.workload}: {prob.nx}x{prob.ny} {dt_name} flux={prob.flux} "
          f"warmup {args.warmup} steps {args.steps}", file=sys.stderr, flush=True)

    if args.warmup > 0:
        st.run(W, A, args.warmup)
    W.copy_(W0)
    A.copy_(A0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t_sim, fail = st.run(W, A, args.steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    # a run that meets a non-physical state skips its later steps: count the steps that ran
    done = args.steps if fail == -1 else fail
    if fail != -1:
        print(f"# non-physical state after {fail} steps: only those are counted", file=sys.stderr)
    cells = prob.nx * prob.ny
    value = cells * done / elapsed
    print(f"# timed {args.steps} steps in {elapsed * 1e3:.2f} ms -> {value:.4e} cell-updates/s (t_sim {t_sim:.5f})",
          file=sys.stderr, flush=True)

    roofline = None
    kernels = None
    if not args.no_profile:
        W.copy_(W0)
        A.copy_(A0)
        torch.cuda.synchronize()
        with api.KernelProfile() as kp:
            st.run(W, A, args.steps)
        prof = kp.result()
        kernels = {k: {"avg_us": 1e3 * ms / n if n else None, "launches": n, "total_ms": ms}
                   for k, (ms, n) in prof.items()}
    # the exact flop count covers the interface kernel of eq. (21) without the limiter; the other
    # forms report times only
    if not args.no_profile and default_form:
        ms1, n1 = prof["faces1"]
        avg_s = ms1 / n1 / 1e3
        faces = (prob.nx + 1) * prob.ny + prob.nx * (prob.ny + 1)
        fl = faces * flops.per_interface(prob.flux, 1)
        achieved = fl / avg_s / 1e12
        peak = PEAK_FP64_VALU if esize == 8 else PEAK_FP32_VALU
        roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                    "frac": round(achieved / peak, 4),
                    "traffic": load_traffic(f"traffic_faces1_{args.workload}.json"),
                    "kernel": "k_faces (first stage)", "flops_per_launch": fl, "avg_launch_us": round(avg_s * 1e6, 2),
                    "flops_counted": "arithmetic the kernel executes: adds, multiplies, divides, sqrt, exp, erfc "
                                     "of its own device functions counted on the host, operations the compiler "
                                     "folds excluded"}
        print(f"# faces1 avg {avg_s * 1e6:.1f} us -> {achieved:.2f} TFLOP/s", file=sys.stderr, flush=True)

    hbm = BYTES_PER_CELL_UPDATE[esize] * value / 1e9
    out = {
        "metric": "cell-updates/s per S2O4 step" if not ts else "cell-updates/s per SSP-RK3 step",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dt_name,
        "data": "synthetic",
        "config": {"workload": workload_text(prob, tl, ts),
                   "name": args.workload, "nx": prob.nx, "ny": prob.ny, "flux": "gks" if prob.flux else "lf",
                   "time_scheme": "ssprk3" if ts else "s2o4", "time_limiter": bool(tl), "tile": params.tile,
                   "parallelism": "single GPU"},
        "fail_step": fail,
        "roofline": roofline,
        "hbm_algorithmic": {"bytes_per_cell_update": BYTES_PER_CELL_UPDATE[esize], "achieved_GBps": round(hbm, 1),
                            "peak_GBps": PEAK_HBM, "frac": round(hbm / PEAK_HBM, 4)} if default_form else None,
        "flops_per_cell_update": flops.per_cell_update(prob.flux) if default_form else None,
        "kernels": kernels,
        "cpu_baseline": None if args.no_cpu_baseline else cpu_baseline(prob, args.cpu_steps, args.cpu_cells, tl, ts),
        "batched": None if args.no_batch else batch_compare(),
        "batched_f32": None if args.no_batch else batch_compare(dtype_name="f32"),
        "adjoint": None if args.no_adjoint else adjoint_compare(),
        "sharp_edges_lf": None if (args.no_sharp or not args.workload.startswith("circles4096")) else sharp_lf_leg(),
    }
    print(json.dumps(out), flush=True)
    if fail != -1:
        sys.exit(3)


if __name__ == "__main__":
    main()
