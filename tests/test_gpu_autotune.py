"""Every launch configuration of the stored apply (LDS tiles of four shapes,
register-blocked gathers with 1..12 right-hand sides per thread) adds the 81
terms of a site in the same order, so all agree bit for bit; the autotuner
installs one of them."""
import numpy as np
import pytest

import synth
from tests.helpers import dev, log

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dims", [(8, 4, 4, 6), (5, 3, 2, 6), (24, 4, 2, 4), (32, 16, 2, 2)])
@pytest.mark.parametrize("wp,sp,noff", [(0, 0, 80), (1, 1, 80), (1, 1, 40), (2, 1, 80), (2, 2, 80)])
def test_all_configurations_bitwise_equal(dims, wp, sp, noff):
    import torch
    import paper_1012_3615_amd as bri
    from paper_1012_3615_amd import autotune
    u = synth.gauge_links(dims, 0.3, 61)
    psi = synth.gaussian_spinor(dims, 62, nrhs=12)
    U = bri.bri_pack_links(dims, dev(u), bri.F64)
    W = bri.bri_build_transporters(dims, U, wp, noff)
    x = bri.bri_pack_spinor(dims, dev(psi), sp)
    old = (bri.bri_get_apply_kernel(wp, sp), bri.bri_get_rhs_block(wp, sp))
    outs = {}
    try:
        for name, kernel, rblk in autotune.candidates(dims, 12, sp) + [("default", 1, 1)]:
            log(f"config {name} dims={dims} w={wp} s={sp} noff={noff}")
            bri.bri_set_apply_kernel(wp, sp, kernel)
            bri.bri_set_rhs_block(wp, sp, rblk)
            outs[name] = (bri.bri_apply(dims, W, x, 0.1).cpu(), bri.bri_apply_dag(dims, W, x, 0.1).cpu())
    finally:
        bri.bri_set_apply_kernel(wp, sp, old[0])
        bri.bri_set_rhs_block(wp, sp, old[1])
    ref = outs["default"]
    for name, (o, od) in outs.items():
        assert torch.equal(o, ref[0]) and torch.equal(od, ref[1]), name


def test_autotuner_installs_a_configuration(tmp_path, monkeypatch):
    import paper_1012_3615_amd as bri
    from paper_1012_3615_amd import autotune
    monkeypatch.setattr(autotune, "CACHE", str(tmp_path / "tune.json"))
    dims = (8, 8, 8, 8)
    u = synth.gauge_links(dims, 0.3, 63)
    psi = synth.gaussian_spinor(dims, 64, nrhs=12)
    log("autotune 8^4 12 rhs")
    U = bri.bri_pack_links(dims, dev(u), bri.F64)
    W = bri.bri_build_transporters(dims, U, bri.F32, 80)
    x = bri.bri_pack_spinor(dims, dev(psi), bri.F32)
    old = (bri.bri_get_apply_kernel(1, 1), bri.bri_get_rhs_block(1, 1))
    try:
        name, ms, table = autotune.tune(dims, W, x)
        assert name in table and ms == min(table.values())
        again = autotune.tune(dims, W, x)          # served from the cache
        assert again[0] == name
        kernel = bri.bri_get_apply_kernel(1, 1)
        assert name.startswith(autotune.TILES.get(kernel, "gather"))
        autotune.reset(1, 1)
        assert (bri.bri_get_apply_kernel(1, 1), bri.bri_get_rhs_block(1, 1)) == (1, 2)
    finally:
        bri.bri_set_apply_kernel(1, 1, old[0])
        bri.bri_set_rhs_block(1, 1, old[1])
