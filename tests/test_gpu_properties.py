"""Properties of the GPU output that hold at any size: free plane waves are
eigenvectors with the closed-form symbol (Eq. def_4Dbri, App. C), pure-gauge
links act like the free field on gauge-rotated constants, and the largest
lattice tested (48^3 x 96: transporter planes indexed past 2^31 elements)
matches the pointwise oracle at sampled sites."""
import numpy as np
import pytest

import synth
from oracle import dirac, free
from tests.helpers import dev, host, log, soa_to_canon

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("mom", [(0, 0, 0, 0), (1, 2, 0, 3), (4, 4, 4, 8), (3, 1, 5, 2)])
def test_plane_waves_on_gpu(mom):
    import paper_1012_3615_amd as bri
    dims = (8, 8, 8, 16)
    u = synth.unit_links(dims)
    rng = np.random.default_rng(8)
    chi = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
    psi = synth.plane_wave(dims, mom, chi)[None]
    k = 2 * np.pi * np.array(mom) / np.array(dims)
    expect = synth.plane_wave(dims, mom, free.symbol(k, 0.1) @ chi)
    log(f"plane wave {mom}")
    U = bri.bri_pack_links(dims, dev(u), bri.F64)
    for wp, sp, tol in [(0, 0, 1e-13), (1, 1, 1e-5)]:
        W = bri.bri_build_transporters(dims, U, wp, 80)
        out = soa_to_canon(dims, bri.bri_apply(dims, W, bri.bri_pack_spinor(dims, dev(psi), sp), 0.1))[0]
        assert np.linalg.norm(out - expect) / np.linalg.norm(psi) < tol


def test_pure_gauge_constant_on_gpu():
    import paper_1012_3615_amd as bri
    dims = (8, 4, 6, 8)
    g = synth.random_su3_field(dims, 81)
    u = synth.gauge_transform_links(synth.unit_links(dims), g)
    v = (np.arange(12).reshape(4, 3) + 1) * (0.3 - 0.7j)
    const = np.broadcast_to(v, synth.lattice_shape(dims) + (4, 3)).copy()
    gv = synth.gauge_transform_spinor(const, g)[None]
    log("pure gauge constant")
    U = bri.bri_pack_links(dims, dev(u), bri.F64)
    W = bri.bri_build_transporters(dims, U, bri.F64, 40)
    out = soa_to_canon(dims, bri.bri_apply(dims, W, bri.bri_pack_spinor(dims, dev(gv), bri.F64), 0.25))
    assert np.linalg.norm(out - 0.25 * gv) / np.linalg.norm(gv) < 1e-13


def test_largest_lattice_sampled():
    import torch
    import paper_1012_3615_amd as bri
    dims = (48, 48, 48, 96)
    log("48^3x96 FP16-W apply, sampled sites")
    Ud = synth.gauge_links_device(dims, 0.3, 4801)
    U = bri.bri_pack_links(dims, Ud, bri.F64)
    psi = torch.complex(torch.randn(synth.lattice_shape(dims) + (4, 3), dtype=torch.float64, device="cuda"),
                        torch.randn(synth.lattice_shape(dims) + (4, 3), dtype=torch.float64, device="cuda"))
    psi = psi[None].contiguous()
    W = bri.bri_build_transporters(dims, U, bri.F16, 80)      # 30 GB store
    x = bri.bri_pack_spinor(dims, psi, bri.F32)
    out = bri.bri_unpack_spinor(dims, bri.bri_apply(dims, W, x, 0.1))[0]
    rng = np.random.default_rng(48)
    sites = np.stack([rng.integers(0, L, 64) for L in dims], axis=1)
    sites = np.concatenate([sites, np.array([[47, 47, 47, 95], [0, 0, 0, 0]])])
    # the oracle needs only the links and psi within two sites of each sample
    u_h, p_h = host(Ud), host(psi[0])
    ref = dirac.apply_at(u_h, p_h, 0.1, sites)
    o_h = host(out)
    got = np.stack([o_h[t, z, y, xx] for xx, y, z, t in sites])
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 5e-3
