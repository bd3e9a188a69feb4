"""The flop counts behind the benchmark's roofline figure are those of the kernels' current
arithmetic: a fresh count (the counting scalar run over the kernels' own device functions,
``paper_2402_10914_amd/flops/count.cpp``) equals the stored ``counts.json``, and the per-interface
and per-cell-update figures are composed from it as documented."""
import os

import pytest

from paper_2402_10914_amd import flops


def _have_hipcc():
    return os.path.exists(flops.HIPCC)


@pytest.mark.skipif(not _have_hipcc(), reason="hipcc not available")
def test_stored_counts_match_the_current_arithmetic():
    assert flops.measure() == flops.counts()


def test_per_cell_update_composition():
    c = flops.counts()
    for flux, name in ((0, "lf"), (1, "gks")):
        per = [c["normal_sweep"]["flops"] + c["segment_%s_stage%d" % (name, s)]["flops"] for s in (1, 2)]
        assert flops.per_interface(flux, 1) == per[0] and flops.per_interface(flux, 2) == per[1]
        assert flops.per_cell_update(flux) == 2 * sum(per) + c["update1_per_cell"] + c["update2_per_cell"]
    # the GKS segment holds the LF one's reconstructions and more flux arithmetic
    assert c["segment_gks_stage1"]["flops"] > c["segment_lf_stage1"]["flops"]
