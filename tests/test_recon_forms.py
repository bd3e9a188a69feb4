"""The kernels' reconstruction forms (Section 3.1, eqs. (33)-(39); Section 3.3), run on the host in
FP64 (``tests/recon_forms_check.cpp``): the Gauss-point form used by the tangential sweep equals
the edge polynomial evaluated at the Gauss points, the polynomial keeps the cell average, the
two-coefficient form of the normal sweep equals the full one, the smoothness indicators equal the
Jiang-Shu forms of eq. (38), and cell averages of a quadratic are reconstructed exactly.  These pin
the rewritten arithmetic (candidates through the indicators' differences, the edge value from the
cell mean, the centred Gauss-point evaluation) to the direct definitions, independently of the
GPU."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

BOUNDS = {  # worst deviation relative to max |Q| (indicators: to max |Q|^2)
    "gauss_vs_poly": 1e-13,
    "cell_mean": 1e-13,
    "edge_vs_poly": 1e-13,
    "indicators": 1e-12,
    "quadratic": 1e-13,
}


@pytest.fixture(scope="module")
def worst(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("recon") / "recon_forms_check")
    subprocess.run([HIPCC, "-std=c++17", "-O1", "-x", "hip", "--offload-arch=gfx950",
                    os.path.join(ROOT, "tests", "recon_forms_check.cpp"), "-o", exe], check=True, capture_output=True)
    out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout.splitlines()
    return {ln.split()[0]: float(ln.split()[1]) for ln in out}


@pytest.mark.parametrize("name", sorted(BOUNDS))
def test_reconstruction_form(worst, name):
    assert name in worst, worst
    assert worst[name] < BOUNDS[name], (name, worst[name])
