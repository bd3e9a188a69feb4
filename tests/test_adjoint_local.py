"""The hand-written adjoints of the device arithmetic (basis, projections, WENO-AO/DF
reconstruction, DF factor, LF and GKS fluxes, normal sweep, Gauss-point segment) against central
differences of the same forward functions, run on the host (CPU)."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def lines(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("adj") / "adjoint_check")
    subprocess.run([HIPCC, "-std=c++17", "-O1", "-x", "hip", "--offload-arch=gfx950",
                    os.path.join(ROOT, "tests", "adjoint_check.cpp"), "-o", exe], check=True, capture_output=True)
    out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout.splitlines()
    return [ln.split() for ln in out]


def test_every_adjoint_matches_central_differences(lines):
    names = {ln[0] for ln in lines}
    for need in ("project", "unproject", "recon5_weno", "recon5_df", "recon2_weno", "recon2_df", "recon_gauss_weno",
                 "recon_gauss_df", "df_factor",
                 "lf_flux", "gks_flux", "gks_flux_tau0", "normal_sweep", "normal_sweep_df", "segment_lf",
                 "segment_lf_df", "segment_gks", "segment_gks_df", "normal_side_fwd", "normal_side_fwd_df"):
        assert need in names, need
    worst = max(lines, key=lambda ln: float(ln[1]))
    assert float(worst[1]) < 1e-6, worst
