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
    outs = {}
    try:
        for name, kernel, rblk in autotune.candidates(dims, 12, sp) + [("default", -1, 0)]:
            log(f"config {name} dims={dims} w={wp} s={sp} noff={noff}")
            bri.bri_set_apply_config(dims, wp, sp, noff, 12, kernel, rblk)
            outs[name] = (bri.bri_apply(dims, W, x, 0.1).cpu(), bri.bri_apply_dag(dims, W, x, 0.1).cpu())
    finally:
        bri.bri_clear_apply_configs()
    ref = outs["default"]
    for name, (o, od) in outs.items():
        assert torch.equal(o, ref[0]) and torch.equal(od, ref[1]), name


def test_autotuner_installs_a_configuration(tmp_path, monkeypatch):
    """A 12-RHS tune installs its choice for that shape only: a later 1-RHS
    apply on the same lattice and precisions still launches its built-in
    kernel (bit for bit the result from before the tune), with no reset."""
    import torch
    import paper_1012_3615_amd as bri
    from paper_1012_3615_amd import autotune
    monkeypatch.setattr(autotune, "CACHE", str(tmp_path / "tune.json"))
    bri.bri_clear_apply_configs()
    dims = (32, 16, 4, 4)
    u = synth.gauge_links(dims, 0.3, 63)
    psi = synth.gaussian_spinor(dims, 64, nrhs=12)
    log("autotune 32x16x4x4 12 rhs")
    U = bri.bri_pack_links(dims, dev(u), bri.F64)
    W = bri.bri_build_transporters(dims, U, bri.F32, 80)
    x = bri.bri_pack_spinor(dims, dev(psi), bri.F32)
    x1 = x[3:4].contiguous()
    builtin_1 = bri.bri_get_apply_config(dims, 1, 1, 80, 1)
    assert builtin_1 == (13, 1)
    before = bri.bri_apply(dims, W, x1, 0.1).clone()
    try:
        name, ms, table, cached = autotune.tune(dims, W, x)
        assert not cached and name in table and ms == min(table.values())
        again = autotune.tune(dims, W, x)          # served from the cache
        assert again[0] == name and again[3]
        kernel, rblk = bri.bri_get_apply_config(dims, 1, 1, 80, 12)
        assert name.startswith(autotune.TILES.get(kernel, "gather")), (name, kernel, rblk)
        # the single right-hand side shape is untouched by the tune
        assert bri.bri_get_apply_config(dims, 1, 1, 80, 1) == builtin_1
        log("autotune: 1-RHS apply after the 12-RHS tune")
        assert torch.equal(bri.bri_apply(dims, W, x1, 0.1), before)
        # a cache entry made with another library build is not used
        monkeypatch.setattr(autotune, "_lib_digest", "abi0-otherbuild")
        assert not autotune.tune(dims, W, x, reps=1)[3]
    finally:
        bri.bri_clear_apply_configs()
