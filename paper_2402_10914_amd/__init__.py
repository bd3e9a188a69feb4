"""MI355X (gfx950) implementation of one S2O4 time step of the 2-D Euler finite-volume scheme with
the hybrid discontinuity-feedback / WENO-AO reconstruction of Zhang, Ji & Xu (arXiv:2402.10914).

    from paper_2402_10914_amd import Stepper, Params, FLUX_GKS
    st = Stepper(nx, ny, dx, dy, bc_x, bc_y, Params(flux=FLUX_GKS, cfl=0.4))
    t, fail_step = st.run(W, alpha, nsteps)

The C ABI is declared in ``include/dfweno.h``; ``workloads`` builds the seeded synthetic inputs.
Attributes that need torch are imported lazily so that the input generators work without it.
"""

_API = {"Stepper", "Params", "Batch", "Adjoint", "Rollout", "rollout", "KernelProfile", "tile_shapes", "run", "FLUX_LF",
        "FLUX_GKS", "TIME_S2O4", "TIME_SSPRK3", "BC_PERIODIC", "BC_TRANSMISSIVE", "DFWError"}


def __getattr__(name):
    if name in _API:
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
