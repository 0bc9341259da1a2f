"""Parity at the full benchmark sizes, in the launch configuration the
benchmark times (stored transporters, LDS-tiled kernel, one right-hand side),
on outputs the oracle computes site by site: 256 random sites of 32^3 x 64
and 24^3 x 48, for every stored precision and both transporter stores, and
for the recompute variant."""
import numpy as np
import pytest

import synth
from oracle import dirac
from tests.helpers import dev, log

pytestmark = pytest.mark.gpu

TOL = {(0, 0): 1e-12, (1, 1): 1e-5, (2, 1): 5e-3, (2, 2): 5e-3}
_inputs = {}


def inputs(dims, eps, seed):
    key = (dims, eps, seed)
    if key not in _inputs:
        _inputs.clear()
        u = synth.gauge_links(dims, eps, seed)
        psi = synth.gaussian_spinor(dims, seed + 1, nrhs=1)
        rng = np.random.default_rng(seed + 2)
        sites = np.stack([rng.integers(0, L, 256) for L in dims], axis=1)
        # include the lattice corners (every wrap-around direction)
        corners = np.array([[0, 0, 0, 0], [dims[0] - 1, dims[1] - 1, dims[2] - 1, dims[3] - 1],
                            [0, dims[1] - 1, 0, dims[3] - 1]])
        sites = np.concatenate([sites, corners])
        ref = dirac.apply_at(u, psi[0], 0.1, sites)
        _inputs[key] = (u, psi, sites, ref)
    return _inputs[key]


def sampled(bri, dims, out, sites):
    got = bri.bri_unpack_spinor(dims, out).cpu().numpy()[0]
    return np.stack([got[t, z, y, x] for x, y, z, t in sites])


@pytest.mark.parametrize("dims,eps,seed", [((32, 32, 32, 64), 0.3, 4001), ((24, 24, 24, 48), 0.4, 3001)])
def test_fullsize_sampled_parity(dims, eps, seed):
    import torch
    import paper_1012_3615_amd as bri
    u, psi, sites, ref = inputs(dims, eps, seed)
    U = bri.bri_pack_links(dims, dev(u), bri.F64)
    for wp, sp, noff in [(1, 1, 80), (1, 1, 40), (0, 0, 80), (2, 1, 80), (2, 2, 80)]:
        log(f"fullsize {dims} w={wp} s={sp} noff={noff}")
        W = bri.bri_build_transporters(dims, U, wp, noff)
        x = bri.bri_pack_spinor(dims, dev(psi), sp)
        got = sampled(bri, dims, bri.bri_apply(dims, W, x, 0.1), sites)
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        assert err <= TOL[(wp, sp)], (wp, sp, noff, err)
        del W, x
        torch.cuda.empty_cache()
    log(f"fullsize {dims} recompute f32")
    U32 = bri.bri_pack_links(dims, dev(u), bri.F32)
    x = bri.bri_pack_spinor(dims, dev(psi), bri.F32)
    got = sampled(bri, dims, bri.bri_apply(dims, U32, x, 0.1, variant=bri.RECOMPUTE), sites)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= 1e-5
