"""GPU parity of the matrix-core apply (bri_apply_mfma) and its transporter
store (bri_pack_w_mfma) against the FP64 oracle, through the C ABI.

The apply multiplies FP16 operands (transporters times lambda_k or rho_k
normalised to at most 1, each rounded once more after the product, and psi
scaled by a power of two per right-hand side) with FP32 accumulation: three
roundings of u_16 = 4.9e-4 per term, so the relative error of an output
column is ~1e-3 in the 2-norm.  Bars (per right-hand side): 5e-3 in the
2-norm, 1e-2 for the largest element against the column's largest reference
element.  The store itself is the oracle's transporters rounded to FP16:
within half an FP16 unit (2^-11 relative) of each real component.

Lattices cover ragged x-y tiles (the workgroup tile is 4 x 2), extent-2 and
extent-3 directions (the halo wraps onto the tile), t-chunks with a ragged
tail (Lt = 20 with 16-step chunks), right-hand-side counts that fill 1, 2
and 3 column tiles and a partial second block of twelve (13, 25).

The apply reads and writes site-major fields [V, nrhs, 12]; the tests move
the oracle's fields there and back with bri_spinor_to_sites and
bri_spinor_from_sites, whose results are checked bit for bit against a
plain permutation of the SoA tensor."""
import numpy as np
import pytest

import synth
from oracle import dirac, transporters as otr, ultralocal
from tests.helpers import dev, log, plane_offsets, soa_to_canon

pytestmark = pytest.mark.gpu

TOL, TOL_ELEM = 5e-3, 1e-2

CASES = [((4, 4, 4, 4), 12), ((5, 3, 2, 6), 5), ((2, 2, 2, 2), 12), ((6, 4, 4, 8), 13), ((7, 5, 3, 3), 4),
         ((8, 4, 4, 20), 12), ((16, 6, 2, 2), 1), ((4, 2, 3, 4), 25)]


@pytest.fixture(scope="module")
def bri():
    import paper_1012_3615_amd as m
    return m


_cache = {}


def setup_case(dims, nrhs, eps=0.3, seed=5101, mass=0.1):
    key = (dims, nrhs, eps, seed)
    if key not in _cache:
        u = synth.gauge_links(dims, eps, seed)
        psi = synth.gaussian_spinor(dims, seed + 1, nrhs=nrhs)
        ref = np.stack([dirac.apply(u, psi[r], mass) for r in range(nrhs)])
        refd = np.stack([dirac.apply_dag(u, psi[r], mass) for r in range(nrhs)])
        _cache[key] = (u, psi, ref, refd)
    return _cache[key]


def check_columns(got, ref, what, tol=TOL, tol_elem=TOL_ELEM):
    for r in range(ref.shape[0]):
        nr = np.linalg.norm(ref[r])
        if nr == 0.0:
            assert np.all(got[r] == 0.0), f"{what} rhs {r}: nonzero output of a zero column"
            continue
        err = np.linalg.norm(got[r] - ref[r]) / nr
        emax = float(np.abs(got[r] - ref[r]).max() / np.abs(ref[r]).max())
        assert err <= tol and emax <= tol_elem, f"{what} rhs {r}: rel {err:.3e} max-elem {emax:.3e}"


def mfma_apply(bri, dims, Wm, x, mass, bound2=None, **kw):
    """SoA FP32 spinor in, SoA out, through the site-major apply."""
    xs, b2 = bri.bri_spinor_to_sites(dims, x, bound2=True)
    out = bri.bri_apply_mfma(dims, Wm, xs, mass, bound2=b2 if bound2 is None else bound2, **kw)
    return bri.bri_spinor_from_sites(dims, out)


def store_to_canon(dims, Wm):
    """[V, 80, 9, 2] float16 -> complex (80, Lt, Lz, Ly, Lx, 3, 3)."""
    a = Wm.detach().cpu().numpy().astype(np.float64)
    c = a[..., 0] + 1j * a[..., 1]  # [V, 80, 9]
    c = np.transpose(c, (1, 0, 2))   # [80, V, 9]
    return c.reshape((80,) + synth.lattice_shape(dims) + (3, 3))


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (5, 3, 2, 6), (2, 2, 2, 2)])
def test_store_is_rounded_transporters(bri, dims):
    import torch
    u = synth.gauge_links(dims, 0.4, 5201)
    U = bri.bri_pack_links(dims, dev(u), bri.F64)
    offs = plane_offsets(80)
    ref = np.stack([otr.transporter(u, n) for n in offs])
    for prec, noff in [(bri.F64, 80), (bri.F64, 40), (bri.F32, 80), (bri.F32, 40)]:
        log(f"pack store dims={dims} prec={prec} noff={noff}")
        W = bri.bri_build_transporters(dims, U, prec, noff)
        got = store_to_canon(dims, bri.bri_pack_w_mfma(dims, W))
        torch.cuda.synchronize()
        for part in (np.real, np.imag):
            g, r = part(got), part(ref)
            # half an FP16 unit of |r| (|W| <= 1), plus the FP32 source's own rounding
            bound = np.maximum(np.abs(r), 2.0 ** -14) * 2.0 ** -11 * (1 + 1e-3) + 1e-7
            assert np.all(np.abs(g - r) <= bound), (prec, noff, float(np.abs(g - r).max()))


@pytest.mark.parametrize("dims,nrhs", [((4, 4, 4, 4), 12), ((5, 3, 2, 6), 5), ((3, 2, 2, 3), 25), ((7, 5, 3, 3), 1),
                                       ((6, 4, 4, 8), 64)])
def test_site_major_transposes_are_exact(bri, dims, nrhs):
    """The two layouts hold the same numbers: to_sites is the permutation
    [nrhs, 12, V] -> [V, nrhs, 12], from_sites its inverse, bit for bit; the
    bounds are the squared largest |re| or |im| of each right-hand side.
    Shapes cover site counts and component counts (12 nrhs) that are not
    multiples of the 32 x 96 transpose tile."""
    import torch
    V = int(np.prod(dims))
    log(f"site-major transposes dims={dims} nrhs={nrhs}")
    g = torch.Generator(device="cpu").manual_seed(5701 + nrhs)
    x = torch.randn((nrhs, 12, V, 2), generator=g, dtype=torch.float32).cuda()
    x[0] *= 1e-20
    xs, b2 = bri.bri_spinor_to_sites(dims, x, bound2=True)
    assert torch.equal(xs, x.permute(2, 0, 1, 3).contiguous())
    assert torch.equal(b2, torch.amax(x.abs().reshape(nrhs, -1), dim=1).double() ** 2)
    assert torch.equal(bri.bri_spinor_to_sites(dims, x), xs)
    assert torch.equal(bri.bri_spinor_from_sites(dims, xs), x)


@pytest.mark.parametrize("dims,nrhs", CASES)
def test_apply_mfma_matches_oracle(bri, dims, nrhs):
    u, psi, ref, refd = setup_case(dims, nrhs)
    log(f"apply mfma dims={dims} nrhs={nrhs}")
    U = bri.bri_pack_links(dims, dev(u), bri.F64)
    W = bri.bri_build_transporters(dims, U, bri.F32, 80)
    Wm = bri.bri_pack_w_mfma(dims, W)
    x = bri.bri_pack_spinor(dims, dev(psi), bri.F32)
    out = mfma_apply(bri, dims, Wm, x, 0.1)
    outd = mfma_apply(bri, dims, Wm, x, 0.1, dagger=True)
    check_columns(soa_to_canon(dims, out), ref, "D")
    check_columns(soa_to_canon(dims, outd), refd, "D^dag")


@pytest.mark.parametrize("name", ["wilson", "hypercube", "random"])
def test_apply_mfma_coefficient_tables(bri, name):
    dims, nrhs = (6, 4, 4, 8), 6
    table = {"wilson": ultralocal.WILSON, "hypercube": ultralocal.HYPERCUBE,
             "random": tuple(float(v) for v in np.random.default_rng(8401).uniform(-1.0, 1.0, 9))}[name]
    u = synth.gauge_links(dims, 0.3, 5301)
    psi = synth.gaussian_spinor(dims, 5302, nrhs=nrhs)
    ref = np.stack([ultralocal.apply(u, psi[r], 0.1, table) for r in range(nrhs)])
    refd = np.stack([ultralocal.apply_dag(u, psi[r], 0.1, table) for r in range(nrhs)])
    log(f"apply mfma table={name}")
    U = bri.bri_pack_links(dims, dev(u), bri.F64)
    Wm = bri.bri_pack_w_mfma(dims, bri.bri_build_transporters(dims, U, bri.F64, 40))
    x = bri.bri_pack_spinor(dims, dev(psi), bri.F32)
    check_columns(soa_to_canon(dims, mfma_apply(bri, dims, Wm, x, 0.1, coef=table)), ref, f"D {name}")
    check_columns(soa_to_canon(dims, mfma_apply(bri, dims, Wm, x, 0.1, dagger=True, coef=table)), refd,
                  f"D^dag {name}")


def test_brillouin_table_equals_default(bri):
    import torch
    dims = (6, 4, 4, 8)
    u = synth.gauge_links(dims, 0.3, 5401)
    psi = synth.gaussian_spinor(dims, 5402, nrhs=12)
    log("apply mfma brillouin table vs default")
    U = bri.bri_pack_links(dims, dev(u), bri.F64)
    Wm = bri.bri_pack_w_mfma(dims, bri.bri_build_transporters(dims, U, bri.F32, 80))
    x = bri.bri_pack_spinor(dims, dev(psi), bri.F32)
    a = mfma_apply(bri, dims, Wm, x, 0.1)
    b = mfma_apply(bri, dims, Wm, x, 0.1, coef=bri.TABLE_BRILLOUIN)
    assert torch.equal(a, b)


def test_column_scales_are_independent(bri):
    """Columns 1e-30, 1, 1e30 times a Gaussian field and an all-zero column
    in one launch: each column keeps its own relative accuracy (the FP16
    operand of psi is scaled per right-hand side), the zero column stays
    exactly zero."""
    import torch
    dims = (6, 4, 4, 8)
    u = synth.gauge_links(dims, 0.3, 5501)
    psi = synth.gaussian_spinor(dims, 5502, nrhs=5)
    psi[0] *= 1e-30
    psi[2] *= 1e30
    psi[3] = 0.0
    psi[4] *= 1e-6
    ref = np.stack([dirac.apply(u, psi[r], 0.1) for r in range(5)])
    log("apply mfma column scales")
    U = bri.bri_pack_links(dims, dev(u), bri.F64)
    Wm = bri.bri_pack_w_mfma(dims, bri.bri_build_transporters(dims, U, bri.F64, 80))
    x = bri.bri_pack_spinor(dims, dev(psi), bri.F32)
    b2 = bri.bri_spinor_bound2(dims, x)
    want = torch.amax(x.abs().reshape(5, -1), dim=1).double() ** 2
    assert torch.equal(b2, want)
    check_columns(soa_to_canon(dims, mfma_apply(bri, dims, Wm, x, 0.1, bound2=b2)), ref, "scaled columns")
    # a loose bound (the squared 2-norm) gives the same accuracy
    n2 = (x.double() ** 2).reshape(5, -1).sum(dim=1)
    check_columns(soa_to_canon(dims, mfma_apply(bri, dims, Wm, x, 0.1, bound2=n2)), ref, "2-norm bound")


def test_apply_mfma_rejects_bad_arguments(bri):
    import torch
    dims = (4, 4, 4, 4)
    V = 256
    Wm = torch.zeros((V, 80, 9, 2), dtype=torch.float16, device="cuda")
    x = torch.zeros((V, 2, 12, 2), dtype=torch.float32, device="cuda")
    b2 = torch.ones(2, dtype=torch.float64, device="cuda")
    lib = bri.api._lib_handle
    D = bri.api._dims(dims)
    assert lib.bri_apply_mfma(D, Wm.data_ptr(), 0.1, x.data_ptr(), x.data_ptr(), 2, 0, None, b2.data_ptr(),
                              None) == -1  # in and out overlap
    out = torch.empty_like(x)
    assert lib.bri_apply_mfma(D, Wm.data_ptr(), 0.1, x.data_ptr(), out.data_ptr(), 2, 2, None, b2.data_ptr(),
                              None) == -1  # dagger not 0/1
    assert lib.bri_apply_mfma(D, Wm.data_ptr(), 0.1, x.data_ptr(), out.data_ptr(), 0, 0, None, b2.data_ptr(),
                              None) == -1  # nrhs
    assert lib.bri_apply_mfma(D, Wm.data_ptr(), 0.1, x.data_ptr(), out.data_ptr(), 2, 0, None, None,
                              None) == -1  # no bound
    assert lib.bri_apply_mfma(D, Wm.data_ptr(), 0.1, x.data_ptr(), out.data_ptr(), 2, 0, None, b2.data_ptr(),
                              None) == 0
    torch.cuda.synchronize()
    assert torch.count_nonzero(out) == 0
    # the layout conversions: overlap and right-hand-side count
    assert lib.bri_spinor_to_sites(D, 2, x.data_ptr(), x.data_ptr(), None, None) == -1
    assert lib.bri_spinor_from_sites(D, 2, x.data_ptr(), x.data_ptr(), None) == -1
    assert lib.bri_spinor_to_sites(D, 0, x.data_ptr(), out.data_ptr(), None, None) == -1
    assert lib.bri_spinor_from_sites(D, 70000, x.data_ptr(), out.data_ptr(), None) == -1


def test_mixed_solve_with_matrix_core_inner_apply(bri):
    """Twelve point sources solved to a true FP64 residual of 1e-10 with the
    FP16 matrix-core apply in the inner CGNE; the FP64 outer loop sees the
    exact operator, so the solution matches the plain FP64 solve."""
    import torch
    dims = (8, 8, 4, 8)
    u = synth.gauge_links(dims, 0.3, 5601)
    b = np.zeros((12,) + synth.lattice_shape(dims) + (4, 3), dtype=np.complex128)
    for s in range(4):
        for c in range(3):
            b[3 * s + c, 0, 0, 0, 0, s, c] = 1.0
    log("mixed solve, matrix-core inner apply")
    U = bri.bri_pack_links(dims, dev(u), bri.F64)
    W_hi = bri.bri_build_transporters(dims, U, bri.F64, 40)
    Wm = bri.bri_pack_w_mfma(dims, W_hi)
    bs = bri.bri_pack_spinor(dims, dev(b), bri.F64)
    p = bri.solve_params(tol=1e-10, inner_tol=1e-2, n_offsets=40, inner_prec=bri.F16, inner_mfma=True)
    x, info = bri.bri_solve_cgne(dims, W_hi, bs, 0.1, p, W_lo=Wm)
    assert info["converged"] and max(info["true_residual"][:12]) <= 1e-10, info
    p64 = bri.solve_params(tol=1e-10, n_offsets=40)
    x64, info64 = bri.bri_solve_cgne(dims, W_hi, bs, 0.1, p64)
    assert info64["converged"]
    rel = float(torch.linalg.norm(x - x64) / torch.linalg.norm(x64))
    assert rel < 1e-8, rel
    # the same with D^dag
    pd = bri.solve_params(tol=1e-10, inner_tol=1e-2, n_offsets=40, inner_prec=bri.F16, inner_mfma=True,
                          dagger=True)
    xd, infod = bri.bri_solve_cgne(dims, W_hi, bs, 0.1, pd, W_lo=Wm)
    assert infod["converged"] and max(infod["true_residual"][:12]) <= 1e-10, infod


@pytest.mark.parametrize("nrhs", [1, 5, 43])
def test_mixed_solve_matrix_core_rhs_counts(bri, nrhs):
    """The site-major inner CGNE with right-hand-side counts that leave the
    BLAS-1 workgroups partly idle (5: 240 of 256 threads; 43: one site per
    pass) and a partial block of twelve in the apply: Gaussian sources, true
    FP64 residual 1e-10, solution equal to the plain FP64 solve."""
    import torch
    dims = (6, 4, 4, 8)
    u = synth.gauge_links(dims, 0.3, 5701)
    src = synth.gaussian_spinor(dims, 5702, nrhs=nrhs)
    log(f"mixed solve, matrix-core inner apply, nrhs={nrhs}")
    U = bri.bri_pack_links(dims, dev(u), bri.F64)
    W_hi = bri.bri_build_transporters(dims, U, bri.F64, 80)
    Wm = bri.bri_pack_w_mfma(dims, W_hi)
    bs = bri.bri_pack_spinor(dims, dev(src), bri.F64)
    p = bri.solve_params(tol=1e-10, inner_tol=1e-2, inner_prec=bri.F16, inner_mfma=True)
    x, info = bri.bri_solve_cgne(dims, W_hi, bs, 0.1, p, W_lo=Wm)
    assert info["converged"] and max(info["true_residual"][:nrhs]) <= 1e-10, info
    x64, info64 = bri.bri_solve_cgne(dims, W_hi, bs, 0.1, bri.solve_params(tol=1e-10))
    rel = float(torch.linalg.norm(x - x64) / torch.linalg.norm(x64))
    assert rel < 1e-8, rel
