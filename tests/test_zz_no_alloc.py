"""dfw_run_noalloc (the entry point for callers that cannot allocate device memory) through the C
ABI against dfw_run on the same inputs: two calls in a row on one GPU, the second on a smaller grid
(the fixed scratch array keeps the first call's contents), FP64 and FP32, and a grid beyond the
array's size rejected before any launch."""
import ctypes

import numpy as np
import pytest

from paper_2402_10914_amd import workloads as WL

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _noalloc(pr, params, dtype, nsteps):
    from paper_2402_10914_amd import _lib, api
    L = _lib.load()
    W = torch.tensor(pr.W, dtype=dtype, device="cuda")
    A = torch.tensor(pr.alpha, dtype=dtype, device="cuda")
    dth = torch.zeros(max(nsteps, 1), dtype=torch.float64, device="cuda")
    g = _lib.dfw_grid(pr.nx, pr.ny, pr.dx, pr.dy, pr.bc_x, pr.bc_y)
    p = params.struct()
    t = ctypes.c_double(0.0)
    fs = ctypes.c_int32(-7)
    st = L.dfw_run_noalloc(ctypes.c_void_p(W.data_ptr()), ctypes.c_void_p(A.data_ptr()), ctypes.byref(g),
                           ctypes.byref(p), nsteps, api._dtype_code(dtype), ctypes.c_void_p(dth.data_ptr()),
                           ctypes.byref(t), ctypes.byref(fs),
                           ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    _lib.check(st)
    torch.cuda.synchronize()
    return W.double().cpu().numpy(), A.double().cpu().numpy(), t.value, fs.value, dth.cpu().numpy()


def _with_ws(pr, params, dtype, nsteps):
    from paper_2402_10914_amd import api
    st = api.Stepper.for_problem(pr, params, dtype)
    W = torch.tensor(pr.W, dtype=dtype, device="cuda")
    A = torch.tensor(pr.alpha, dtype=dtype, device="cuda")
    dth = torch.zeros(max(nsteps, 1), dtype=torch.float64, device="cuda")
    t, fs = st.run(W, A, nsteps, dt_hist=dth)
    torch.cuda.synchronize()
    return W.double().cpu().numpy(), A.double().cpu().numpy(), t, fs, dth.cpu().numpy()


def _rel_l1(a, b):
    a, b = np.atleast_3d(a), np.atleast_3d(b)
    return max(float(np.abs(a[c] - b[c]).sum() / np.abs(b[c]).sum()) for c in range(a.shape[0]))


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("flux", [WL.FLUX_LF, WL.FLUX_GKS])
def test_noalloc_matches_run_on_two_calls(flux, dtype):
    from paper_2402_10914_amd import api
    params = api.Params(flux=flux, cfl=0.4)
    # first call on the largest grid the array holds in FP64, second on a smaller ragged grid
    for pr, nsteps in ((WL.riemann4(512, seed=2402), 6), (WL.riemann4(37, 23, seed=5), 9)):
        got = _noalloc(pr, params, dtype, nsteps)
        ref = _with_ws(pr, params, dtype, nsteps)
        assert got[3] == -1 and ref[3] == -1
        # the same kernels on the same inputs: bitwise equal, far inside the parity bound
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
        assert _rel_l1(got[0], ref[0]) <= (1e-12 if dtype == torch.float64 else 1e-5)
        assert got[2] == ref[2]
        np.testing.assert_array_equal(got[4], ref[4])


def test_noalloc_rejects_grids_beyond_the_array():
    from paper_2402_10914_amd import _lib, api
    L = _lib.load()
    g = _lib.dfw_grid(1024, 1024, 1e-3, 1e-3, 0, 0)
    assert L.dfw_workspace_bytes(ctypes.byref(g), _lib.DFW_F64) > _lib.DFW_NOALLOC_SCRATCH_BYTES
    W = torch.ones(4, 1024, 1024, dtype=torch.float64, device="cuda")
    A = torch.ones(1024, 1024, dtype=torch.float64, device="cuda")
    p = api.Params(cfl=0.4).struct()
    fs = ctypes.c_int32(-7)
    st = L.dfw_run_noalloc(ctypes.c_void_p(W.data_ptr()), ctypes.c_void_p(A.data_ptr()), ctypes.byref(g),
                           ctypes.byref(p), 1, _lib.DFW_F64, None, None, ctypes.byref(fs),
                           ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == _lib.DFW_EWORKSPACE
    assert b"scratch" in L.dfw_last_error()
    assert fs.value == -7  # nothing ran
    assert bool((W == 1).all())
