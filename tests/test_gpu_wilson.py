"""GPU parity of the Wilson comparison operator (Sec. 1; the Wilson column
of Tab. rholambda) applied straight from the links, against the oracle's
generic-class apply with the Wilson table (pinned against the hopping form
of the Wilson operator in the oracle tests).

Tolerances as for the Brillouin operator: FP64 1e-12, FP32 1e-5 (relative
2-norm against the FP64 oracle); at 32^3 x 64 on sampled sites."""
import numpy as np
import pytest

import synth
from oracle import ultralocal
from oracle.gamma import gamma5
from tests.helpers import dev, log, soa_to_canon

pytestmark = pytest.mark.gpu

TOL = {0: 1e-12, 1: 1e-5}


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def bri():
    import paper_1012_3615_amd as m
    return m


# L = 2 in a direction (forward and backward neighbour coincide), odd
# extents, a volume that is not a multiple of the 256-site workgroup; Lx a
# multiple of 32 and Ly of 8 take the LDS-tiled kernel (one tile in y, so
# the y halo wraps onto the tile itself; two tiles in x and y), with two z
# slices per workgroup where Lz is even and one where it is odd
@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (6, 5, 3, 4), (2, 3, 2, 5), (16, 6, 2, 2), (32, 8, 2, 3),
                                  (64, 16, 2, 2), (32, 8, 3, 2), (32, 8, 4, 3)])
def test_wilson_matches_oracle(bri, dims):
    mass = 0.1
    u = synth.gauge_links(dims, 0.4, 8701)
    psi = synth.gaussian_spinor(dims, 8702, nrhs=3)
    want = np.stack([ultralocal.apply(u, psi[r], mass, ultralocal.WILSON) for r in range(3)])
    want_dag = np.stack([ultralocal.apply_dag(u, psi[r], mass, ultralocal.WILSON) for r in range(3)])
    for p in (0, 1):
        log(f"wilson {dims} prec={p}")
        U = bri.bri_pack_links(dims, dev(u), p)
        for nr in (1, 3):
            x = bri.bri_pack_spinor(dims, dev(psi[:nr]), p)
            got = soa_to_canon(dims, bri.bri_apply_wilson(dims, U, x, mass))
            gdg = soa_to_canon(dims, bri.bri_apply_wilson(dims, U, x, mass, dagger=True))
            for r in range(nr):
                assert rel(got[r], want[r]) < TOL[p], (p, nr, r)
                assert rel(gdg[r], want_dag[r]) < TOL[p], (p, nr, r, "dag")


def test_wilson_gamma5_hermiticity_and_free_field(bri):
    """D_W^dag = gamma5 D_W gamma5 on random links; on unit links a plane wave
    e^{ik.x} u is mapped to the Wilson symbol times u (momenta allowed by the
    periodic lattice)."""
    dims = (8, 4, 6, 4)
    mass = 0.05
    u = synth.gauge_links(dims, 0.4, 8703)
    psi = synth.gaussian_spinor(dims, 8704, nrhs=1)
    U = bri.bri_pack_links(dims, dev(u), bri.F64)
    x = bri.bri_pack_spinor(dims, dev(psi), bri.F64)
    g5psi = np.einsum("st,...tc->...sc", gamma5(), psi)
    x5 = bri.bri_pack_spinor(dims, dev(g5psi), bri.F64)
    dag = soa_to_canon(dims, bri.bri_apply_wilson(dims, U, x, mass, dagger=True))[0]
    g5dg5 = np.einsum("st,...tc->...sc", gamma5(), soa_to_canon(dims, bri.bri_apply_wilson(dims, U, x5, mass))[0])
    assert rel(dag, g5dg5) < 1e-13
    # free field
    lx, ly, lz, lt = dims
    k = 2 * np.pi * np.array([1 / lx, 2 / ly, 1 / lz, 3 / lt])
    t, z, y, xx = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx), indexing="ij")
    ph = np.exp(1j * (k[0] * xx + k[1] * y + k[2] * z + k[3] * t))
    rng = np.random.default_rng(8705)
    spin = rng.normal(size=(4, 3)) + 1j * rng.normal(size=(4, 3))
    wave = ph[..., None, None] * spin
    unit = np.zeros_like(u)
    unit[..., 0, 0] = unit[..., 1, 1] = unit[..., 2, 2] = 1
    Uu = bri.bri_pack_links(dims, dev(unit), bri.F64)
    got = soa_to_canon(dims, bri.bri_apply_wilson(dims, Uu, bri.bri_pack_spinor(dims, dev(wave[None]), bri.F64),
                                                  mass))[0]
    sym = ultralocal.fourier_sum(k, mass, ultralocal.WILSON)
    want = ph[..., None, None] * np.einsum("st,tc->sc", sym, spin)
    assert rel(got, want) < 1e-13


def test_wilson_full_size_sampled(bri):
    """32^3 x 64, FP32, one right-hand side, the launch the bench times:
    64 random sites (and the eight corners) against the pointwise oracle."""
    dims = (32, 32, 32, 64)
    mass = 0.1
    log("wilson 32^3x64 sampled")
    u = synth.gauge_links(dims, 0.3, 4001)
    psi = synth.gaussian_spinor(dims, 4002, nrhs=1)
    U = bri.bri_pack_links(dims, dev(u), bri.F32)
    x = bri.bri_pack_spinor(dims, dev(psi), bri.F32)
    got = soa_to_canon(dims, bri.bri_apply_wilson(dims, U, x, mass))[0]
    rng = np.random.default_rng(8706)
    sites = np.stack([rng.integers(0, L, 64) for L in dims], axis=1)
    corners = np.array([[a * (dims[0] - 1), b * (dims[1] - 1), 0, c * (dims[3] - 1)]
                        for a in (0, 1) for b in (0, 1) for c in (0, 1)])
    sites = np.concatenate([sites, corners])
    want = ultralocal.apply_at(u, psi[0], mass, ultralocal.WILSON, sites)
    g = np.stack([got[t, z, y, xx] for xx, y, z, t in sites])
    assert rel(g, want) < TOL[1]


def test_wilson_t_chunks_with_ragged_tail(bri):
    """Enough work for the t walk to run in chunks of 8 (32^3 x 12, twelve
    right-hand sides): chunks [0, 8) and [8, 12), so the carried backward hop
    crosses a chunk start and the last chunk is short; FP64, D and D^dag, on
    sampled sites including every t slice next to a chunk edge."""
    dims = (32, 32, 32, 12)
    mass = 0.1
    log("wilson 32^3x12 12 rhs chunks")
    u = synth.gauge_links(dims, 0.3, 8707)
    psi = synth.gaussian_spinor(dims, 8708, nrhs=12)
    U = bri.bri_pack_links(dims, dev(u), bri.F64)
    x = bri.bri_pack_spinor(dims, dev(psi), bri.F64)
    got = soa_to_canon(dims, bri.bri_apply_wilson(dims, U, x, mass))
    gdg = soa_to_canon(dims, bri.bri_apply_wilson(dims, U, x, mass, dagger=True))
    rng = np.random.default_rng(8709)
    ts = np.array([0, 7, 8, 11, 3, 9])
    sites = np.stack([rng.integers(0, 32, 12), rng.integers(0, 32, 12), rng.integers(0, 32, 12),
                      np.repeat(ts, 2)], axis=1)
    for r in range(12):
        want = ultralocal.apply_at(u, psi[r], mass, ultralocal.WILSON, sites)
        g = np.stack([got[r, t, z, y, xx] for xx, y, z, t in sites])
        assert rel(g, want) < TOL[0], r
    # D^dag at the same sites from gamma5 D gamma5 of the oracle (whole-lattice
    # adjoint would be slow at this size)
    g5 = gamma5()
    psi5 = np.einsum("st,...tc->...sc", g5, psi[0])
    want = np.einsum("st,...tc->...sc", g5, ultralocal.apply_at(u, psi5, mass, ultralocal.WILSON, sites))
    g = np.stack([gdg[0, t, z, y, xx] for xx, y, z, t in sites])
    assert rel(g, want) < TOL[0]


def test_wilson_rejects_bad_arguments(bri):
    import torch
    dims = (4, 4, 4, 4)
    U = torch.zeros((4, 9, 256, 2), dtype=torch.float16, device="cuda")
    x = torch.zeros((1, 12, 256, 2), dtype=torch.float16, device="cuda")
    with pytest.raises(Exception):
        bri.bri_apply_wilson(dims, U, x, 0.1)
    U = torch.zeros((4, 9, 256, 2), dtype=torch.float32, device="cuda")
    x = torch.zeros((1, 12, 256, 2), dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        bri.bri_apply_wilson(dims, U, x, 0.1)


def test_matched_low_end_iterations(bri):
    """The spectral argument behind the paper's iteration counts (Sec. 6,
    footnote): with the Wilson mass tuned so that the smallest eigenvalue of
    D^dag D matches the Brillouin one, the largest is several times larger
    for Wilson (near 7.5^2 against 2.5^2), and CGNE on the Brillouin operator
    needs well under half the iterations.  8^4, links eps 0.3; Wilson through
    the generic-class table (same solver and store)."""
    import torch
    dims = (8, 8, 8, 8)
    log("wilson vs brillouin matched low end 8^4")
    U = bri.bri_pack_links(dims, dev(synth.gauge_links(dims, 0.3, 8711)), bri.F64)
    W = bri.bri_build_transporters(dims, U, bri.F64, 80)
    opb, opw = bri.Operator(W), bri.Operator(W, coef=bri.TABLE_WILSON)
    b = bri.bri_pack_spinor(dims, dev(synth.gaussian_spinor(dims, 8712, nrhs=1)), bri.F64)
    v0 = bri.bri_pack_spinor(dims, dev(synth.gaussian_spinor(dims, 8713, nrhs=1)), bri.F64)

    def extremes(op, m):
        a, bb, _ = bri.bri_lanczos(dims, op, m, 120, v0)
        r = bri.bri_ritz_values(a, bb)
        return float(r[0]), float(r[-1])

    m_b = 0.1
    lo_b, hi_b = extremes(opb, m_b)
    m_w = m_b
    for _ in range(4):
        lo_w, _ = extremes(opw, m_w)
        m_w += float(np.sqrt(lo_b) - np.sqrt(lo_w))
    lo_w, hi_w = extremes(opw, m_w)
    assert abs(lo_w / lo_b - 1) < 1e-3
    assert hi_w / hi_b > 8
    p = bri.solve_params(tol=1e-10, inner_prec=bri.F64)
    _, ib = bri.bri_solve_cgne_op(dims, opb, b, m_b, p)
    _, iw = bri.bri_solve_cgne_op(dims, opw, b, m_w, p)
    assert ib["true_residual"][0] < 1e-10 and iw["true_residual"][0] < 1e-10
    assert ib["iterations"] < 0.5 * iw["iterations"], (ib["iterations"], iw["iterations"])
    torch.cuda.synchronize()
