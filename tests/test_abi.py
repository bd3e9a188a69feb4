"""The C ABI library loads on the host, exports every entry point that include/*.h declares, its
structs match the header, and argument validation works without touching a GPU."""
import ctypes
import glob
import os
import re
import subprocess

import pytest

from paper_2402_10914_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = []
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        txt = open(h).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(dfw_[a-z0-9_]+)\s*\(", txt, re.M):
            names.append(m.group(1))
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    L = _lib.load()
    names = _declared_functions()
    assert "dfw_run" in names and "dfw_rhs" in names
    for n in names:
        assert hasattr(L, n), n
    assert set(names) <= set(_lib.SIGNATURES), set(names) - set(_lib.SIGNATURES)


def test_struct_layout_matches_header(tmp_path):
    src = tmp_path / "probe.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "dfweno.h"\nint main(void){'
                   'printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(dfw_grid), offsetof(dfw_grid, dx),'
                   ' offsetof(dfw_grid, bc_y), sizeof(dfw_params), offsetof(dfw_params, c2),'
                   ' offsetof(dfw_params, tile), offsetof(dfw_params, time_limiter),'
                   ' offsetof(dfw_params, time_scheme), offsetof(dfw_params, t_end),'
                   ' offsetof(dfw_params, switch_rule), offsetof(dfw_params, df_stage)); return 0;}\n')
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    want = [ctypes.sizeof(_lib.dfw_grid), _lib.dfw_grid.dx.offset, _lib.dfw_grid.bc_y.offset,
            ctypes.sizeof(_lib.dfw_params), _lib.dfw_params.c2.offset, _lib.dfw_params.tile.offset,
            _lib.dfw_params.time_limiter.offset, _lib.dfw_params.time_scheme.offset, _lib.dfw_params.t_end.offset,
            _lib.dfw_params.switch_rule.offset, _lib.dfw_params.df_stage.offset]
    assert out == want


def _grid(nx=8, ny=8):
    return _lib.dfw_grid(nx, ny, 0.1, 0.1, 0, 0)


def _params(**kw):
    d = dict(gamma=1.4, cfl=0.5, dt_fixed=0.0, alpha_thres=0.5, d_h=0.85, d_l=0.85, eps_weno=1e-6, c1=0.01, c2=5.0,
             flux=0, tile=0, time_limiter=0, time_scheme=0, t_end=0.0, switch_rule=0, componentwise=0,
             df_stage=0)
    d.update(kw)
    return _lib.dfw_params(*[d[k] for k, _ in _lib.dfw_params._fields_])


def test_workspace_bytes_host_only():
    L = _lib.load()
    g = _grid(100, 50)
    b64 = L.dfw_workspace_bytes(ctypes.byref(g), 0)
    b32 = L.dfw_workspace_bytes(ctypes.byref(g), 1)
    n = 100 * 50
    assert b64 >= 8 * (8 * n + 9 * (50 * 101 + 51 * 100))
    assert b32 < b64
    assert L.dfw_workspace_bytes(ctypes.byref(_grid(0, 5)), 0) == 0


@pytest.mark.parametrize("case,status", [
    (dict(grid=_grid(0, 4)), _lib.DFW_EINVAL),
    (dict(params=_params(gamma=1.0)), _lib.DFW_EINVAL),
    (dict(params=_params(flux=7)), _lib.DFW_EINVAL),
    (dict(params=_params(cfl=0.0, dt_fixed=0.0)), _lib.DFW_EINVAL),
    (dict(params=_params(tile=99)), _lib.DFW_EINVAL),
    (dict(params=_params(time_limiter=2)), _lib.DFW_EINVAL),
    (dict(params=_params(time_scheme=2)), _lib.DFW_EINVAL),
    (dict(params=_params(time_scheme=1, flux=1)), _lib.DFW_EINVAL),  # SSP-RK3 runs with LF only
    (dict(params=_params(time_scheme=1, time_limiter=1)), _lib.DFW_EINVAL),
    (dict(params=_params(t_end=-1.0)), _lib.DFW_EINVAL),
    (dict(params=_params(switch_rule=3)), _lib.DFW_EINVAL),
    (dict(params=_params(componentwise=2)), _lib.DFW_EINVAL),
    (dict(params=_params(df_stage=-1)), _lib.DFW_EINVAL),
    (dict(dtype=5), _lib.DFW_EDTYPE),
    (dict(W=None), _lib.DFW_EINVAL),
    (dict(nsteps=-1), _lib.DFW_EINVAL),
    (dict(ws=None), _lib.DFW_EWORKSPACE),
    (dict(ws=257), _lib.DFW_EWORKSPACE),
    (dict(ws_bytes=16), _lib.DFW_EWORKSPACE),
])
def test_run_validation_without_gpu(case, status):
    L = _lib.load()
    a = dict(W=4096, alpha=8192, grid=_grid(), params=_params(), nsteps=1, dtype=0, ws=1 << 20, ws_bytes=1 << 30)
    a.update(case)
    st = L.dfw_run(a["W"], a["alpha"], ctypes.byref(a["grid"]), ctypes.byref(a["params"]), a["nsteps"], a["dtype"],
                   a["ws"], a["ws_bytes"], None, None, None, None)
    assert st == status
    assert len(L.dfw_last_error()) > 0


def test_rhs_and_speed_validation_without_gpu():
    L = _lib.load()
    g, p = _grid(), _params()
    assert L.dfw_rhs(4096, 8192, ctypes.byref(g), ctypes.byref(p), 0, 0.0, 4096, 4096, None, 1 << 20, 1 << 30,
                     None) == _lib.DFW_EINVAL
    assert L.dfw_max_speed(None, ctypes.byref(g), ctypes.byref(p), 0, 1 << 20, 1 << 30, None, None,
                           None) == _lib.DFW_EINVAL


def test_full_tape_sizes_without_gpu():
    """ckpt_every = 1 keeps each step's whole record (W^n, alpha^n, W*, the stage-2 DF products of
    the x and the y interfaces, each region 256-byte aligned) and no recomputation buffers."""
    L = _lib.load()
    nx, ny, n = 37, 23, 5
    g = _grid(nx, ny)
    a = lambda b: (b + 255) // 256 * 256
    N, sx, sy = nx * ny, ny * (nx + 1), (ny + 1) * nx
    rec = a(4 * N * 8) + a(N * 8) + a(4 * N * 8) + a(sx * 8) + a(sy * 8)
    assert L.dfw_checkpoint_bytes(ctypes.byref(g), 0, n, 1) == n * rec
    assert L.dfw_checkpoint_bytes(ctypes.byref(g), 0, n, 2) == 3 * (a(4 * N * 8) + a(N * 8))
    ws1 = L.dfw_adjoint_workspace_bytes(ctypes.byref(g), 0, 1)
    ws2 = L.dfw_adjoint_workspace_bytes(ctypes.byref(g), 0, 2)
    assert ws2 - ws1 == 2 * (2 * a(4 * N * 8) + a(N * 8) + a(sx * 8) + a(sy * 8))


def test_adjoint_validation_without_gpu():
    """dfw_adjoint validates before any device work: FP32, the time limiter, a missing dt history
    and a small checkpoint store are rejected; the size queries are host-only."""
    L = _lib.load()
    g = _grid(16, 12)
    n, every = 7, 3
    ck = L.dfw_checkpoint_bytes(ctypes.byref(g), 0, n, every)
    ws = L.dfw_adjoint_workspace_bytes(ctypes.byref(g), 0, every)
    assert ck > 0 and ws > 0
    assert L.dfw_checkpoint_bytes(ctypes.byref(g), 0, n, 0) == 0
    assert L.dfw_checkpoint_bytes(ctypes.byref(g), 0, n, 4) < ck  # fewer segments
    def call(params, dtype=0, dt_hist=4096, ckpt_bytes=ck):
        return L.dfw_adjoint(ctypes.byref(g), ctypes.byref(params), dtype, n, every, 1 << 20, ckpt_bytes, dt_hist,
                             4096, None, 8192, None, 1 << 24, ws, None)
    assert call(_params(), dtype=1) == _lib.DFW_EDTYPE
    assert call(_params(time_limiter=1)) == _lib.DFW_EINVAL
    assert call(_params(time_scheme=1)) == _lib.DFW_EINVAL
    assert call(_params(t_end=0.5)) == _lib.DFW_EINVAL
    assert call(_params(componentwise=1)) == _lib.DFW_EINVAL
    assert call(_params(df_stage=1)) == _lib.DFW_EINVAL
    assert call(_params(), dt_hist=None) == _lib.DFW_EINVAL
    assert call(_params(), ckpt_bytes=ck - 1) == _lib.DFW_EINVAL
    assert L.dfw_run_ckpt(4096, 8192, ctypes.byref(g), ctypes.byref(_params()), n, 0, 0, 1 << 20, ck, 1 << 24,
                          1 << 30, 4096, None, None, None) == _lib.DFW_EINVAL  # ckpt_every = 0


def _host_stepper(nx=8, ny=6):
    """A Stepper whose arguments are checked without a GPU (no workspace, no library calls)."""
    import torch
    from paper_2402_10914_amd import _lib, api
    st = api.Stepper.__new__(api.Stepper)
    st.grid = _lib.dfw_grid(nx, ny, 0.1, 0.1, 0, 0)
    st.params = api.Params()
    st.dtype = torch.float64
    st.device = torch.device("cuda", 0)
    st.lib = None  # any library call would fail: the checks must raise first
    return st


def test_host_tensors_are_rejected_before_any_launch():
    """Host tensors, strided views and mismatched dt_hist raise ValueError in the binding, so no
    host pointer or strided view reaches a kernel."""
    import torch
    from paper_2402_10914_amd import api
    st = _host_stepper()
    W = torch.zeros(4, 6, 8, dtype=torch.float64)
    A = torch.ones(6, 8, dtype=torch.float64)
    with pytest.raises(ValueError, match="W must be"):
        st.run(W, A, 1)
    with pytest.raises(ValueError, match="W must be"):
        st.run(torch.zeros(4, 8, 6, dtype=torch.float64).transpose(1, 2), A, 1)
    with pytest.raises(ValueError, match="W must be"):
        st.max_speed(W)
    with pytest.raises(ValueError):
        st.rhs(W, A, 1e-3)
    b = api.Batch.__new__(api.Batch)
    b.ngrids, b.w_elems, b.a_elems = 2, 40, 10
    b.dtype, b.device, b.lib, b.handle = torch.float64, torch.device("cuda", 0), None, None
    with pytest.raises(ValueError, match="packed W"):
        b.run(torch.zeros(40, dtype=torch.float64), torch.zeros(10, dtype=torch.float64), 1)
    with pytest.raises(ValueError, match="packed W"):
        b.run(torch.zeros(80, dtype=torch.float64)[::2], torch.zeros(10, dtype=torch.float64), 1)
