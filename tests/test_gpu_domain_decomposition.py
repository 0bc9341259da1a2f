"""The sharding design on one GPU: the lattice is cut into sub-domains along
z and t ("ranks" inside one process); each rank receives its slab plus a
depth-1 halo of links and spinors on every cut side, corners included (what
the per-dimension exchange delivers), builds its own transporters and
applies the operator on the extended slab; the interior of every rank must
equal the single-domain result bit for bit.  This holds because every
transporter of an interior site, and every intermediate one it is built
from, depends only on links inside the hypercube between its two end points,
which lies within the halo."""
import numpy as np
import pytest

import synth
from tests.helpers import dev, log

pytestmark = pytest.mark.gpu


def _ext(a, axis, lo, hi, L):
    """Slab [lo, hi) along `axis` plus one halo layer on each side (periodic)."""
    return np.take(a, np.arange(lo - 1, hi + 1) % L, axis=axis)


@pytest.mark.parametrize("split", [(1, 2), (2, 2), (1, 4), (4, 1)])
@pytest.mark.parametrize("prec", [0, 1])
def test_subdomains_match_single_domain(split, prec):
    import paper_1012_3615_amd as bri
    dims = (8, 4, 4, 8)
    lx, ly, lz, lt = dims
    nzp, ntp = split
    u = synth.gauge_links(dims, 0.3, 9101)
    psi = synth.gaussian_spinor(dims, 9102, nrhs=2)
    log(f"domain decomposition split z={nzp} t={ntp} prec={prec}")
    U = bri.bri_pack_links(dims, dev(u), bri.F64)
    W = bri.bri_build_transporters(dims, U, prec, 80)
    ref = bri.bri_unpack_spinor(dims, bri.bri_apply(dims, W, bri.bri_pack_spinor(dims, dev(psi), prec), 0.1))
    ref = ref.cpu().numpy()
    bz, bt = lz // nzp, lt // ntp
    for iz in range(nzp):
        for it in range(ntp):
            z0, t0 = iz * bz, it * bt
            # links [4, Lt, Lz, Ly, Lx, 3, 3]; spinors [rhs, Lt, Lz, Ly, Lx, 4, 3]
            ue = _ext(_ext(u, 1, t0, t0 + bt, lt), 2, z0, z0 + bz, lz)
            pe = _ext(_ext(psi, 1, t0, t0 + bt, lt), 2, z0, z0 + bz, lz)
            de = (lx, ly, bz + 2, bt + 2)
            Ue = bri.bri_pack_links(de, dev(ue), bri.F64)
            We = bri.bri_build_transporters(de, Ue, prec, 80)
            oe = bri.bri_unpack_spinor(de, bri.bri_apply(de, We, bri.bri_pack_spinor(de, dev(pe), prec), 0.1))
            interior = oe.cpu().numpy()[:, 1:-1, 1:-1]
            assert np.array_equal(interior, ref[:, t0:t0 + bt, z0:z0 + bz]), (iz, it)
