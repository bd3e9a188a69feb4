"""Exact arithmetic counts of the HIP formulation (see count.cpp), used as the algorithmic flops of
the roofline report.  ``counts()`` reads counts.json; ``regenerate()`` rebuilds it with hipcc."""
from __future__ import annotations

import json
import os
import subprocess
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
JSON = os.path.join(HERE, "counts.json")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def measure() -> dict:
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "count")
        subprocess.run([HIPCC, "-std=c++17", "-O1", "-x", "hip", "--offload-arch=gfx950",
                        os.path.join(HERE, "count.cpp"), "-o", exe], check=True, capture_output=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    return json.loads(out)


def regenerate() -> dict:
    c = measure()
    with open(JSON, "w") as f:
        json.dump(c, f, indent=1)
        f.write("\n")
    return c


def counts() -> dict:
    with open(JSON) as f:
        return json.load(f)


def per_interface(flux: int, stage: int) -> int:
    """Flops of one interface segment (normal sweep + tangential sweep + two Gauss-point fluxes)."""
    c = counts()
    seg = c["segment_%s_stage%d" % ("gks" if flux == 1 else "lf", stage)]["flops"]
    return c["normal_sweep"]["flops"] + seg


def per_cell_update(flux: int) -> int:
    """Flops of one cell advanced by one S2O4 step (two interfaces per cell per stage)."""
    c = counts()
    return 2 * (per_interface(flux, 1) + per_interface(flux, 2)) + c["update1_per_cell"] + c["update2_per_cell"]


if __name__ == "__main__":
    print(json.dumps(regenerate(), indent=1))
