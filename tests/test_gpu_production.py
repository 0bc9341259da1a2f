"""GPU parity of the production-operator path (Sec. 5) against the oracle:
SU(3) projection, APE smearing, back-projected transporters in both stores,
the clover term, the full operator and its adjoint in every precision, and
the solver on it.

Tolerances: FP64 1e-12 (relative 2-norm; the projection's Newton refinement
and the SVD route differ between the two sides only by rounding), FP32
1e-5, FP16 transporter storage 5e-3.  For the projection of raw matrices the
bound is per matrix, 1e-13 + 1e-15 kappa^2 with kappa = s_max/s_min: the GPU
takes the singular values from the eigenvalues of A^dag A, whose rounding
error relative to the smallest one grows like kappa^2 (path averages and APE
arguments have kappa < 10)."""
import numpy as np
import pytest

import synth
from oracle import clover as oclover
from oracle import production, projection, smearing
from oracle.lattice import all_offsets
from oracle.transporters import make_site_getter
from tests.helpers import dev, host, log, soa_to_canon

pytestmark = pytest.mark.gpu

TOL = {(0, 0): 1e-12, (1, 1): 1e-5, (2, 1): 5e-3, (2, 2): 5e-3}


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def bri():
    import paper_1012_3615_amd as m
    return m


def _mats_to_soa(a):
    """(n, 3, 3) complex -> FP64 tensor [9, n, 2]."""
    import torch
    n = a.shape[0]
    c = a.reshape(n, 9).T
    return torch.from_numpy(np.ascontiguousarray(np.stack([c.real, c.imag], axis=-1))).cuda()


def _soa_to_mats(t):
    a = host(t)
    c = a[..., 0] + 1j * a[..., 1]
    return c.T.reshape(-1, 3, 3)


def _test_matrices(seed, n):
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((n, 3, 3)) + 1j * rng.standard_normal((n, 3, 3))
    s1 = synth.random_su3_field((n, 1, 1, 1), seed + 1).reshape(n, 3, 3)
    s2 = synth.random_su3_field((n, 1, 1, 1), seed + 2).reshape(n, 3, 3)
    near = s1 + 0.05 * (rng.standard_normal((n, 3, 3)) + 1j * rng.standard_normal((n, 3, 3)))
    b = 2.0
    foot = np.eye(3) + np.diag([np.exp(1j * b), np.exp(1j * b), np.exp(-2j * b)])
    return np.concatenate([g, 0.5 * (s1 + s2), near, foot[None]])


def test_project_su3_matches_oracle(bri):
    a = _test_matrices(7001, 1000)        # 3001 matrices: several blocks and a ragged tail
    log(f"project_su3 n={a.shape[0]}")
    want = projection.project_sun(a)
    sv = np.linalg.svd(a, compute_uv=False)
    kappa = sv[:, 0] / sv[:, 2]
    bound = 1e-13 + 1e-15 * kappa ** 2
    A = _mats_to_soa(a)
    got = _soa_to_mats(bri.bri_project_su3(A))
    err = np.abs(got - want).reshape(len(a), -1).max(axis=1)
    assert np.all(err <= bound), (err.max(), kappa[np.argmax(err / bound)])
    assert err[kappa < 10].max() < 1e-13
    # in place, and SU(3) inputs come back unchanged
    bri.bri_project_su3(A, out=A)
    assert np.all(np.abs(_soa_to_mats(A) - want).reshape(len(a), -1).max(axis=1) <= bound)
    u = synth.random_su3_field((257, 1, 1, 1), 7002).reshape(-1, 3, 3)
    assert np.abs(_soa_to_mats(bri.bri_project_su3(_mats_to_soa(u))) - u).max() < 1e-13
    assert bri.bri_project_su3(_mats_to_soa(a[:0])).shape == (9, 0, 2)


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (5, 3, 4, 6)])
def test_ape_matches_oracle(bri, dims):
    log(f"ape {dims}")
    u = synth.gauge_links(dims, 0.4, 7101)
    want = smearing.ape(u, 0.72)
    U = bri.bri_pack_links(dims, dev(u), bri.F64)
    got = host(bri.bri_unpack_links(dims, bri.bri_ape_smear(dims, U, 0.72)))
    assert rel(got, want) < 1e-12
    assert np.abs(host(bri.bri_unpack_links(dims, bri.bri_ape_smear(dims, U, 0.0))) - u).max() < 1e-14


def _w_plane_canon(dims, W, j, rows):
    """Plane j of a transporter store as complex (Lt,Lz,Ly,Lx,rows,3)."""
    a = host(W[j]).astype(np.float64)
    c = a[..., 0] + 1j * a[..., 1]            # [3*rows, V]
    return c.T.reshape(synth.lattice_shape(dims) + (rows, 3))


@pytest.mark.parametrize("noff", [80, 40])
def test_projected_transporters_match_oracle(bri, noff):
    dims = (4, 3, 4, 5)
    log(f"projected transporters noff={noff}")
    u = synth.gauge_links(dims, 0.4, 7201)
    U = bri.bri_pack_links(dims, dev(u), bri.F64)
    W3 = bri.bri_build_transporters_ex(dims, U, bri.F64, noff, bri.W_SU3)
    W2 = bri.bri_build_transporters_ex(dims, U, bri.F64, noff, bri.W_SU3_2ROW)
    W3f = bri.bri_build_transporters_ex(dims, U, bri.F32, noff, bri.W_SU3)
    offs = all_offsets()                      # index i = (nx+1) + 3(ny+1) + 9(nz+1) + 27(nt+1), 40 skipped
    for j in range(noff):
        i = (j if j < 40 else j + 1) if noff == 80 else j + 41
        n = offs[i if i < 40 else i - 1]
        want = production.transporter_su3(u, n)
        assert np.abs(_w_plane_canon(dims, W3, j, 3) - want).max() < 1e-12, (j, n)
        assert np.abs(_w_plane_canon(dims, W2, j, 2) - want[..., :2, :]).max() < 1e-12, (j, n)
        assert np.abs(_w_plane_canon(dims, W3f, j, 3) - want).max() < 1e-6, (j, n)


def _decode_clover(dims, C):
    """[2,18,V,2] -> two Hermitian 6x6 blocks per site, complex (Lt,Lz,Ly,Lx,2,6,6)."""
    a = host(C).astype(np.float64)
    c = a[..., 0] + 1j * a[..., 1]            # [2, 18, V]
    V = c.shape[2]
    m = np.zeros((2, V, 6, 6), dtype=np.complex128)
    for b in range(2):
        for p in range(3):
            m[b, :, 2 * p, 2 * p] = c[b, p].real
            m[b, :, 2 * p + 1, 2 * p + 1] = c[b, p].imag
        q = 3
        for i in range(6):
            for j in range(i + 1, 6):
                m[b, :, i, j] = c[b, q]
                m[b, :, j, i] = np.conj(c[b, q])
                q += 1
    return np.transpose(m, (1, 0, 2, 3)).reshape(synth.lattice_shape(dims) + (2, 6, 6))


def test_clover_term_matches_oracle(bri):
    dims = (4, 5, 3, 4)
    log("clover build and apply")
    u = synth.gauge_links(dims, 0.5, 7301)
    U = bri.bri_pack_links(dims, dev(u), bri.F64)
    full = oclover.clover_matrix(u, 1.0)      # (..., 12, 12)
    C = bri.bri_build_clover(dims, U, 1.0, bri.F64)
    blocks = _decode_clover(dims, C)
    assert np.abs(blocks[..., 0, :, :] - full[..., :6, :6]).max() < 1e-13
    assert np.abs(blocks[..., 1, :, :] - full[..., 6:, 6:]).max() < 1e-13
    assert np.abs(full[..., :6, 6:]).max() == 0 and np.abs(full[..., 6:, :6]).max() == 0
    # applied: (D with clover) - (D without) = clover term
    psi = synth.gaussian_spinor(dims, 7302, nrhs=2)
    W = bri.bri_build_transporters(dims, U, bri.F64, 80)
    x = bri.bri_pack_spinor(dims, dev(psi), bri.F64)
    with_c = bri.bri_apply_op(dims, bri.Operator(W, bri.W_AVERAGE, C), x, 0.1)
    without = bri.bri_apply(dims, W, x, 0.1)
    diff = soa_to_canon(dims, with_c - without)
    for r in range(2):
        assert rel(diff[r], oclover.apply_clover(u, psi[r], 1.0)) < 1e-12


PREC = [(0, 0), (1, 1), (2, 1), (2, 2)]


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (32, 12, 2, 2), (24, 10, 2, 2), (2, 3, 2, 2)])
def test_production_operator_matches_oracle(bri, dims):
    """Smeared links, two-row SU(3) transporters and clover term, D and D^dag,
    one and three right-hand sides, every precision pair; (32,12,2,2) runs the
    32x8 tile and (24,10,2,2) the 24x8 tile, each with a partial tile in y."""
    import torch
    mass = 0.1
    u = synth.gauge_links(dims, 0.4, 7401)
    psi = synth.gaussian_spinor(dims, 7402, nrhs=3)
    us = smearing.ape(u, 0.72)
    want = np.stack([production.apply(us, psi[r], mass) for r in range(3)])
    want_dag = np.stack([production.apply_dag(us, psi[r], mass) for r in range(3)])
    U = bri.bri_pack_links(dims, dev(u), bri.F64)
    Us = bri.bri_ape_smear(dims, U, 0.72)
    for wp, sp in PREC:
        for form in (bri.W_SU3_2ROW, bri.W_SU3):
            log(f"production {dims} w={wp} s={sp} form={form}")
            W = bri.bri_build_transporters_ex(dims, Us, wp, 80, form)
            C = bri.bri_build_clover(dims, Us, 1.0, sp)
            op = bri.Operator(W, form, C)
            for nr in (1, 3):
                x = bri.bri_pack_spinor(dims, dev(psi[:nr]), sp)
                got = soa_to_canon(dims, bri.bri_apply_op(dims, op, x, mass))
                gdg = soa_to_canon(dims, bri.bri_apply_op(dims, op, x, mass, dagger=True))
                for r in range(nr):
                    assert rel(got[r], want[r]) <= TOL[(wp, sp)], (wp, sp, form, nr, r)
                    assert rel(gdg[r], want_dag[r]) <= TOL[(wp, sp)], (wp, sp, form, nr, r, "dag")
            del W, C
            torch.cuda.empty_cache()


def test_production_rejects_unsupported(bri):
    dims = (4, 4, 4, 4)
    U = bri.bri_pack_links(dims, dev(synth.gauge_links(dims, 0.3, 7501)), bri.F64)
    W40 = bri.bri_build_transporters_ex(dims, U, bri.F32, 40, bri.W_SU3_2ROW)
    x = bri.bri_pack_spinor(dims, dev(synth.gaussian_spinor(dims, 7502, nrhs=1)), bri.F32)
    with pytest.raises(bri.BriError, match="n_offsets = 80"):
        bri.bri_apply_op(dims, bri.Operator(W40, bri.W_SU3_2ROW), x, 0.1)


@pytest.mark.parametrize("inner", [0, 1, 2])
def test_production_solve(bri, inner):
    """CGNE on the production operator to 1e-10: plain FP64 and defect
    correction with FP32 / FP16 transporters (FP32 clover); the true residual
    is recomputed with the oracle."""
    dims, mass = (4, 4, 4, 4), 0.2
    u = synth.gauge_links(dims, 0.4, 7601)
    b = synth.gaussian_spinor(dims, 7602, nrhs=2)
    log(f"production solve inner={inner}")
    U = bri.bri_ape_smear(dims, bri.bri_pack_links(dims, dev(u), bri.F64), 0.72)
    hi = bri.Operator(bri.bri_build_transporters_ex(dims, U, bri.F64, 80, bri.W_SU3_2ROW), bri.W_SU3_2ROW,
                      bri.bri_build_clover(dims, U, 1.0, bri.F64))
    lo = None
    if inner:
        lo = bri.Operator(bri.bri_build_transporters_ex(dims, U, inner, 80, bri.W_SU3_2ROW), bri.W_SU3_2ROW,
                          bri.bri_build_clover(dims, U, 1.0, bri.F32))
    p = bri.solve_params(tol=1e-10, inner_tol=1e-3 if inner == 1 else 1e-2, inner_prec=inner)
    B = bri.bri_pack_spinor(dims, dev(b), bri.F64)
    X, info = bri.bri_solve_cgne_op(dims, hi, B, mass, p, op_lo=lo)
    assert info["converged"] and max(info["true_residual"]) <= 1e-10
    xs = soa_to_canon(dims, X)
    us = smearing.ape(u, 0.72)
    for r in range(2):
        res = production.apply(us, xs[r], mass) - b[r]
        assert np.linalg.norm(res) / np.linalg.norm(b[r]) <= 2e-10


_FULL = {}


def _smeared_near(u, sites, dims):
    """APE-smeared links on the union of the 3^4 neighbourhoods of the sampled
    sites (NaN elsewhere, so any use of a missing entry shows)."""
    off = np.array(np.meshgrid(*[np.arange(-1, 2)] * 4, indexing="ij")).reshape(4, -1).T
    near = (sites[:, None, :] + off[None, :, :]).reshape(-1, 4) % np.array(dims)
    near = np.unique(near, axis=0)
    get = make_site_getter(near, dims)
    vs = np.full(u.shape, np.nan + 0j)
    for mu in range(4):
        v = smearing.ape_link(u, mu, 0.72, get)
        vs[mu][near[:, 3], near[:, 2], near[:, 1], near[:, 0]] = v
    return vs


@pytest.mark.parametrize("dims", [(24, 24, 24, 48), (32, 16, 4, 4)])
def test_production_fullsize_sampled(bri, dims):
    """24^3 x 48 (eps = 0.4, the mixed-solve lattice; 24x8 tiles) and
    32x16x4x4 (32x8 tiles with Ly a multiple of 16): 64 random sites plus
    corners, FP64 and FP32 two-row transporters with the clover term."""
    import torch
    mass = 0.1
    log(f"production sampled {dims}: host inputs")
    u = synth.gauge_links(dims, 0.4, 3001)
    psi = synth.gaussian_spinor(dims, 3002, nrhs=1)
    rng = np.random.default_rng(7701)
    sites = np.stack([rng.integers(0, L, 64) for L in dims], axis=1)
    sites = np.concatenate([sites, [[0, 0, 0, 0], [d - 1 for d in dims]]])
    vs = _smeared_near(u, sites, dims)
    want = production.apply_at(vs, psi[0], mass, sites)
    assert np.isfinite(want).all()
    U = bri.bri_ape_smear(dims, bri.bri_pack_links(dims, dev(u), bri.F64), 0.72)
    for wp, sp in [(0, 0), (1, 1)]:
        log(f"production sampled {dims} w={wp} s={sp}")
        op = bri.Operator(bri.bri_build_transporters_ex(dims, U, wp, 80, bri.W_SU3_2ROW), bri.W_SU3_2ROW,
                          bri.bri_build_clover(dims, U, 1.0, sp))
        x = bri.bri_pack_spinor(dims, dev(psi), sp)
        got = soa_to_canon(dims, bri.bri_apply_op(dims, op, x, mass))[0]
        g = np.stack([got[t, z, y, xx] for xx, y, z, t in sites])
        assert rel(g, want) <= TOL[(wp, sp)], (wp, sp)
        del op, x
        torch.cuda.empty_cache()


def test_production_twelve_sources_mixed(bri):
    """The 12 spin-colour point sources at 4^4 on the production operator
    (smeared links, two-row SU(3) transporters, clover term), batched mixed
    solve with FP16 transporters inside, to 1e-10; every column's residual
    recomputed with the oracle."""
    dims, mass = (4, 4, 4, 4), 0.1
    u = synth.gauge_links(dims, 0.3, 7801)
    src = synth.point_sources(dims)
    log("production 12-source mixed solve 4^4")
    U = bri.bri_ape_smear(dims, bri.bri_pack_links(dims, dev(u), bri.F64), 0.72)
    hi = bri.Operator(bri.bri_build_transporters_ex(dims, U, bri.F64, 80, bri.W_SU3_2ROW), bri.W_SU3_2ROW,
                      bri.bri_build_clover(dims, U, 1.0, bri.F64))
    lo = bri.Operator(bri.bri_build_transporters_ex(dims, U, bri.F16, 80, bri.W_SU3_2ROW), bri.W_SU3_2ROW,
                      bri.bri_build_clover(dims, U, 1.0, bri.F32))
    p = bri.solve_params(tol=1e-10, inner_tol=1e-2, inner_prec=bri.F16)
    X, info = bri.bri_solve_cgne_op(dims, hi, bri.bri_pack_spinor(dims, dev(src), bri.F64), mass, p, op_lo=lo)
    assert info["converged"] and max(info["true_residual"][:12]) <= 1e-10
    xs = soa_to_canon(dims, X)
    us = smearing.ape(u, 0.72)
    for r in range(12):
        res = production.apply(us, xs[r], mass) - src[r]
        assert np.linalg.norm(res) <= 2e-10 * np.linalg.norm(src[r]), r
