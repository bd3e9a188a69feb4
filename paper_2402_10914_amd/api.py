"""PyTorch-facing API of the S2O4 DF-hybrid step (Zhang, Ji & Xu, arXiv:2402.10914).

PyTorch supplies device memory and the current stream; every step of the method runs in the HIP
kernels of ``libdfweno.so`` through the C ABI of ``include/dfweno.h``.

    st = Stepper(nx, ny, dx, dy, bc_x, bc_y, params=Params(flux=FLUX_GKS, cfl=0.4))
    t, fail_step = st.run(W, alpha, nsteps)     # W [4, ny, nx], alpha [ny, nx], CUDA tensors, in place
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _lib
from ._lib import (DFW_BC_PERIODIC, DFW_BC_TRANSMISSIVE, DFW_ENONPHYS, DFW_F32, DFW_F64, DFW_FLUX_GKS,
                   DFW_FLUX_LF, DFW_OK, DFW_TIME_S2O4, DFW_TIME_SSPRK3, DFWError)

FLUX_LF, FLUX_GKS = DFW_FLUX_LF, DFW_FLUX_GKS
TIME_S2O4, TIME_SSPRK3 = DFW_TIME_S2O4, DFW_TIME_SSPRK3
BC_PERIODIC, BC_TRANSMISSIVE = DFW_BC_PERIODIC, DFW_BC_TRANSMISSIVE


@dataclass
class Params:
    """Scheme parameters; defaults are the paper's (eps_weno is not given by the paper)."""
    flux: int = FLUX_LF
    gamma: float = 1.4
    cfl: float = 0.5
    dt_fixed: float = 0.0
    alpha_thres: float = 0.5
    d_h: float = 0.85
    d_l: float = 0.85
    eps_weno: float = 1e-6
    c1: float = 0.01
    c2: float = 5.0
    tile: int = 0  # interface tile shape (performance only; see tile_shapes())
    time_limiter: int = 0  # 1: non-linear time limiter of Section 2.2, eqs. (27)-(29)
    time_scheme: int = TIME_S2O4  # TIME_SSPRK3: eq. (32) of Section 2.3 (LF flux only)
    t_end: float = 0.0  # > 0: stop at this time (the last step is shortened; nsteps is an upper bound)
    switch_rule: int = 0  # hybrid switch on the max (eq. (42)), 1: min of the three DF values, 2: own cell
    componentwise: int = 0  # 1: reconstruct conservative variables component by component (ablation)
    df_stage: int = 0  # 1: alpha^{n+1} from the first stage's Gauss points (ablation)

    def struct(self) -> _lib.dfw_params:
        return _lib.dfw_params(float(self.gamma), float(self.cfl), float(self.dt_fixed), float(self.alpha_thres),
                               float(self.d_h), float(self.d_l), float(self.eps_weno), float(self.c1),
                               float(self.c2), int(self.flux), int(self.tile), int(self.time_limiter),
                               int(self.time_scheme), float(self.t_end), int(self.switch_rule),
                               int(self.componentwise), int(self.df_stage))


def tile_shapes():
    """[(TF, TR)] of the interface tile shapes the library provides (index = Params.tile)."""
    L = _lib.load()
    out = []
    for k in range(L.dfw_num_tiles()):
        tf, tr = ctypes.c_int32(), ctypes.c_int32()
        _lib.check(L.dfw_tile_shape(k, ctypes.byref(tf), ctypes.byref(tr)))
        out.append((tf.value, tr.value))
    return out


def _dtype_code(dt: torch.dtype) -> int:
    if dt == torch.float64:
        return DFW_F64
    if dt == torch.float32:
        return DFW_F32
    raise TypeError(f"unsupported dtype {dt}; use torch.float64 or torch.float32")


def _stream_ptr(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t: torch.Tensor) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def _same_device(t: torch.Tensor, device: torch.device) -> bool:
    if t.device.type != "cuda":
        return False
    want = device.index if device.index is not None else torch.cuda.current_device()
    return t.device.index == want


def _require(t: torch.Tensor, name: str, dtype: torch.dtype, device: torch.device, numel: int | None = None,
             shape: tuple | None = None, at_least: bool = False):
    """Raises ValueError unless t is a contiguous tensor of `dtype` on the CUDA device `device` with the
    given shape or element count (at least `numel` elements when at_least), so that no host pointer
    and no strided view ever reaches a kernel."""
    ok = isinstance(t, torch.Tensor) and t.dtype == dtype and t.is_contiguous() and _same_device(t, device)
    if ok and shape is not None:
        ok = tuple(t.shape) == tuple(shape)
    if ok and numel is not None:
        ok = t.numel() >= numel if at_least else t.numel() == numel
    if not ok:
        msg = f"{name} must be a contiguous {dtype} tensor on {device}"
        if shape is not None:
            msg += f" of shape {tuple(shape)}"
        if numel is not None:
            msg += f" with {'at least ' if at_least else ''}{numel} elements"
        raise ValueError(msg)


class Stepper:
    """Owns the device workspace for one grid and element type."""

    def __init__(self, nx: int, ny: int, dx: float, dy: float, bc_x: int = BC_PERIODIC, bc_y: int | None = None,
                 params: Params | None = None, dtype: torch.dtype = torch.float64, device="cuda"):
        self.lib = _lib.load()
        self.grid = _lib.dfw_grid(int(nx), int(ny), float(dx), float(dy), int(bc_x),
                                  int(bc_x if bc_y is None else bc_y))
        self.params = params or Params()
        self.dtype = dtype
        self.code = _dtype_code(dtype)
        self.device = torch.device(device)
        nbytes = self.lib.dfw_workspace_bytes(ctypes.byref(self.grid), self.code)
        if nbytes == 0:
            raise DFWError(_lib.DFW_EINVAL, "invalid grid")
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self.ws.data_ptr()) % 256
        self.ws_ptr = ctypes.c_void_p(self.ws.data_ptr() + off)
        self.ws_bytes = nbytes

    @classmethod
    def for_problem(cls, prob, params: Params, dtype=torch.float64, device="cuda"):
        return cls(prob.nx, prob.ny, prob.dx, prob.dy, prob.bc_x, prob.bc_y, params, dtype, device)

    @classmethod
    def tuned(cls, prob, params: Params, dtype=torch.float64, device="cuda"):
        """A Stepper with the interface tile shape the autotuner picks for this grid (timed on the
        problem's own initial state, cached per GPU architecture, sizes and options; results do not
        depend on the tile)."""
        from . import autotune
        tile, _ = autotune.tune_grid(prob, params, dtype)
        return cls.for_problem(prob, Params(**{**params.__dict__, "tile": tile}), dtype, device)

    def _check(self, W: torch.Tensor, alpha: torch.Tensor | None = None):
        g = self.grid
        _require(W, "W", self.dtype, self.device, shape=(4, g.ny, g.nx))
        if alpha is not None:
            _require(alpha, "alpha", self.dtype, self.device, shape=(g.ny, g.nx))

    def run(self, W: torch.Tensor, alpha: torch.Tensor, nsteps: int, dt_hist: torch.Tensor | None = None,
            params: Params | None = None, strict: bool = False):
        """Advance (W, alpha) in place by nsteps time steps (S2O4, or SSP-RK3 when params.time_scheme
        is TIME_SSPRK3).  Returns (t, fail_step); fail_step is -1
        unless a non-physical state was met (then W holds it; strict=True raises instead)."""
        self._check(W, alpha)
        if dt_hist is not None:
            _require(dt_hist, "dt_hist", torch.float64, self.device, numel=nsteps, at_least=True)
        p = (params or self.params).struct()
        t = ctypes.c_double(0.0)
        fs = ctypes.c_int32(-1)
        st = self.lib.dfw_run(_ptr(W), _ptr(alpha), ctypes.byref(self.grid), ctypes.byref(p), int(nsteps), self.code,
                              self.ws_ptr, self.ws_bytes, _ptr(dt_hist) if dt_hist is not None else None,
                              ctypes.byref(t), ctypes.byref(fs), _stream_ptr(self.device))
        if st == DFW_ENONPHYS and not strict:
            return t.value, fs.value
        _lib.check(st)
        return t.value, fs.value

    def max_speed(self, W: torch.Tensor):
        """CFL reduction: (max over cells of max((|U|+c)/dx, (|V|+c)/dy), non-physical flag)."""
        self._check(W)
        s = ctypes.c_double(0.0)
        bad = ctypes.c_int32(0)
        p = self.params.struct()
        _lib.check(self.lib.dfw_max_speed(_ptr(W), ctypes.byref(self.grid), ctypes.byref(p), self.code, self.ws_ptr,
                                          self.ws_bytes, ctypes.byref(s), ctypes.byref(bad),
                                          _stream_ptr(self.device)))
        return s.value, bool(bad.value)

    def rhs(self, W: torch.Tensor, alpha: torch.Tensor, dt: float, want_alpha: bool = False):
        """Spatial operator of one stage: L(W), dL/dt(W) and optionally the DF product per cell."""
        self._check(W, alpha)
        L = torch.empty_like(W)
        Lt = torch.empty_like(W)
        an = torch.empty_like(alpha) if want_alpha else None
        p = self.params.struct()
        _lib.check(self.lib.dfw_rhs(_ptr(W), _ptr(alpha), ctypes.byref(self.grid), ctypes.byref(p), self.code,
                                    float(dt), _ptr(L), _ptr(Lt), _ptr(an) if an is not None else None,
                                    self.ws_ptr, self.ws_bytes, _stream_ptr(self.device)))
        return (L, Lt, an) if want_alpha else (L, Lt)


class Batch:
    """Many independent grids advanced together (one launch per kernel for all grids; optionally
    one hipGraph replay for the whole rollout).  grids: list of (nx, ny, dx, dy, bc_x, bc_y)."""

    def __init__(self, grids, params: Params, dtype: torch.dtype = torch.float64, order: int = 0, device="cuda"):
        self.lib = _lib.load()
        self.ngrids = len(grids)
        arr = (_lib.dfw_grid * self.ngrids)(*[_lib.dfw_grid(int(nx), int(ny), float(dx), float(dy), int(bx), int(by))
                                              for nx, ny, dx, dy, bx, by in grids])
        self.grids = [tuple(g) for g in grids]
        self.params = params
        self.dtype = dtype
        self.code = _dtype_code(dtype)
        self.device = torch.device(device)
        h = ctypes.c_void_p()
        p = params.struct()
        _lib.check(self.lib.dfw_batch_plan(arr, self.ngrids, ctypes.byref(p), self.code, int(order), ctypes.byref(h)))
        self.handle = h
        wo = (ctypes.c_int64 * self.ngrids)()
        ao = (ctypes.c_int64 * self.ngrids)()
        we, ae, wb = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
        _lib.check(self.lib.dfw_batch_layout(h, wo, ao, ctypes.byref(we), ctypes.byref(ae), ctypes.byref(wb)))
        self.w_offsets = list(wo)
        self.a_offsets = list(ao)
        self.w_elems, self.a_elems, self.ws_bytes = we.value, ae.value, wb.value
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        self.ws_ptr = ctypes.c_void_p(self.ws.data_ptr() + (-self.ws.data_ptr()) % 256)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            self.lib.dfw_batch_free(h)
            self.handle = None

    def pack(self, Ws, alphas):
        """Host or device arrays per grid -> packed device tensors (W_flat, alpha_flat)."""
        Wf = torch.empty(self.w_elems, dtype=self.dtype, device=self.device)
        Af = torch.empty(self.a_elems, dtype=self.dtype, device=self.device)
        for g, (nx, ny, *_rest) in enumerate(self.grids):
            n = nx * ny
            Wf[self.w_offsets[g]:self.w_offsets[g] + 4 * n] = torch.as_tensor(Ws[g], dtype=self.dtype).reshape(-1).to(self.device)
            Af[self.a_offsets[g]:self.a_offsets[g] + n] = torch.as_tensor(alphas[g], dtype=self.dtype).reshape(-1).to(self.device)
        return Wf, Af

    def unpack(self, Wf, Af):
        out = []
        for g, (nx, ny, *_rest) in enumerate(self.grids):
            n = nx * ny
            out.append((Wf[self.w_offsets[g]:self.w_offsets[g] + 4 * n].view(4, ny, nx),
                        Af[self.a_offsets[g]:self.a_offsets[g] + n].view(ny, nx)))
        return out

    def run(self, Wf: torch.Tensor, Af: torch.Tensor, nsteps: int, use_graph: bool = True,
            dt_hist: torch.Tensor | None = None):
        """Advance every grid in place.  Returns (t per grid, fail step per grid)."""
        _require(Wf, "packed W", self.dtype, self.device, numel=self.w_elems)
        _require(Af, "packed alpha", self.dtype, self.device, numel=self.a_elems)
        if dt_hist is not None:
            _require(dt_hist, "dt_hist", torch.float64, self.device, numel=self.ngrids * nsteps, at_least=True)
        t = (ctypes.c_double * self.ngrids)()
        fs = (ctypes.c_int32 * self.ngrids)()
        st = self.lib.dfw_batch_run(self.handle, _ptr(Wf), _ptr(Af), int(nsteps), self.ws_ptr, self.ws_bytes,
                                    1 if use_graph else 0, _ptr(dt_hist) if dt_hist is not None else None, t, fs,
                                    _stream_ptr(self.device))
        if st not in (DFW_OK, DFW_ENONPHYS):
            _lib.check(st)
        return list(t), list(fs)


def _aligned_buffer(nbytes: int, device) -> tuple[torch.Tensor, ctypes.c_void_p]:
    buf = torch.empty(max(nbytes, 1) + 256, dtype=torch.uint8, device=device)
    return buf, ctypes.c_void_p(buf.data_ptr() + (-buf.data_ptr()) % 256)


class Adjoint:
    """Checkpointed rollout of one grid and its hand-written adjoint (FP64).

        adj = Adjoint(stepper, nsteps, ckpt_every=10)
        t, fail_step = adj.forward(W, alpha)           # in place; records checkpoints and dt
        gW0, gA0 = adj.backward(gW_N, gA_N)            # dJ/dW^0, dJ/dalpha^0 at the recorded dt

    The time steps are held at the recorded values (the CFL reduction is not differentiated).
    ckpt_every = 1 records each step whole (about 11 values per cell and step: 9.2 GB for 100 steps
    of a 1024 x 1024 grid) and backward recomputes nothing; the gradient is bitwise the same for
    every ckpt_every."""

    def __init__(self, stepper: Stepper, nsteps: int, ckpt_every: int = 10):
        if stepper.dtype != torch.float64:
            raise TypeError("the adjoint is implemented in FP64 only")
        self.st = stepper
        self.lib = stepper.lib
        self.nsteps = int(nsteps)
        self.every = int(ckpt_every)
        g = ctypes.byref(stepper.grid)
        self.ckpt_bytes = self.lib.dfw_checkpoint_bytes(g, stepper.code, self.nsteps, self.every)
        self.ws_bytes = self.lib.dfw_adjoint_workspace_bytes(g, stepper.code, self.every)
        if self.ws_bytes == 0 or self.every < 1 or self.nsteps < 0:
            raise DFWError(_lib.DFW_EINVAL, "invalid adjoint configuration")
        self.ckpt, self.ckpt_ptr = _aligned_buffer(self.ckpt_bytes, stepper.device)
        self.ws, self.ws_ptr = _aligned_buffer(self.ws_bytes, stepper.device)
        self.dt_hist = torch.zeros(max(self.nsteps, 1), dtype=torch.float64, device=stepper.device)
        self.recorded = False

    def forward(self, W: torch.Tensor, alpha: torch.Tensor, params: Params | None = None):
        """Advance (W, alpha) in place by nsteps steps, storing checkpoints.  Returns (t, fail_step)."""
        self.st._check(W, alpha)
        p = (params or self.st.params).struct()
        self.params = p
        t = ctypes.c_double(0.0)
        fs = ctypes.c_int32(-1)
        st = self.lib.dfw_run_ckpt(_ptr(W), _ptr(alpha), ctypes.byref(self.st.grid), ctypes.byref(p), self.nsteps,
                                   self.st.code, self.every, self.ckpt_ptr, self.ckpt_bytes, self.ws_ptr,
                                   self.ws_bytes, _ptr(self.dt_hist), ctypes.byref(t), ctypes.byref(fs),
                                   _stream_ptr(self.st.device))
        if st != DFW_ENONPHYS:
            _lib.check(st)
        self.recorded = st == DFW_OK
        return t.value, fs.value

    def backward(self, gW: torch.Tensor, gA: torch.Tensor | None = None, want_alpha: bool = True):
        """(dJ/dW^N, dJ/dalpha^N or None) -> (dJ/dW^0, dJ/dalpha^0 or None)."""
        if not self.recorded:
            raise RuntimeError("backward needs a successful forward")
        self.st._check(gW, gA)
        gW0 = torch.empty_like(gW)
        gA0 = torch.empty_like(gW[0]) if want_alpha else None
        _lib.check(self.lib.dfw_adjoint(ctypes.byref(self.st.grid), ctypes.byref(self.params), self.st.code,
                                        self.nsteps, self.every, self.ckpt_ptr, self.ckpt_bytes, _ptr(self.dt_hist),
                                        _ptr(gW), _ptr(gA) if gA is not None else None, _ptr(gW0),
                                        _ptr(gA0) if gA0 is not None else None, self.ws_ptr, self.ws_bytes,
                                        _stream_ptr(self.st.device)))
        return gW0, gA0


class Rollout(torch.autograd.Function):
    """(W^N, alpha^N) = Rollout.apply(W0, alpha0, stepper, nsteps, ckpt_every): nsteps S2O4 steps
    whose backward is the hand-written adjoint (checkpoint every ckpt_every steps, dt held at the
    values of the forward).  A non-physical state in the forward raises DFWError."""

    @staticmethod
    def forward(ctx, W0, alpha0, stepper: Stepper, nsteps: int, ckpt_every: int = 10):
        adj = Adjoint(stepper, nsteps, ckpt_every)
        W = W0.detach().clone().contiguous()
        A = alpha0.detach().clone().contiguous()
        _, fs = adj.forward(W, A)
        if fs != -1:
            raise DFWError(DFW_ENONPHYS, f"non-physical state after {fs} steps")
        ctx.adj = adj
        return W, A

    @staticmethod
    def backward(ctx, gW, gA):
        gW0, gA0 = ctx.adj.backward(gW.contiguous(), gA.contiguous() if gA is not None else None)
        return gW0, gA0, None, None, None


def rollout(W0: torch.Tensor, alpha0: torch.Tensor, stepper: Stepper, nsteps: int, ckpt_every: int = 10):
    """Differentiable nsteps rollout: returns (W^N, alpha^N)."""
    return Rollout.apply(W0, alpha0, stepper, nsteps, ckpt_every)


class KernelProfile:
    """Context manager recording the device time of every kernel launched by Stepper.run (HIP
    events on the launch stream); .result() -> {kind: (total_ms, launches)}."""

    def __enter__(self):
        _lib.check(_lib.load().dfw_profile(1))
        return self

    def __exit__(self, *exc):
        self._read()
        _lib.load().dfw_profile(0)
        return False

    def _read(self):
        n = len(_lib.KERNEL_KINDS)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int64 * n)()
        _lib.check(_lib.load().dfw_profile_read(ms, cnt, n))
        self._res = {k: (ms[i], cnt[i]) for i, k in enumerate(_lib.KERNEL_KINDS)}

    def result(self):
        return self._res


def run(W: torch.Tensor, alpha: torch.Tensor, nx_ny_dx_dy_bc, params: Params, nsteps: int):
    """One-shot convenience: ((nx, ny, dx, dy, bc_x, bc_y), ...) -> (t, fail_step)."""
    nx, ny, dx, dy, bcx, bcy = nx_ny_dx_dy_bc
    return Stepper(nx, ny, dx, dy, bcx, bcy, params, W.dtype, W.device).run(W, alpha, nsteps)
