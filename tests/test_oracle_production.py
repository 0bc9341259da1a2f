"""Pins of the production-operator oracle (Sec. 5): the SU(3) projection of
Sec. 5.2, one APE step (Eq. def_ape), the clover term of Eq. def_pref and the
operator with projected transporters.  Each check is independent of the
formula it tests: closed forms from scalar phase arithmetic, group
properties, brute-force optimality, symmetries."""
import itertools

import numpy as np
import pytest

import synth
from oracle import clover, dirac, production, projection, smearing
from oracle.gamma import gamma5, gammas
from oracle.lattice import all_offsets, dag

TOL = 1e-13


def _gauss(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _su3(n, seed):
    return synth.random_su3_field((n, 1, 1, 1), seed).reshape(n, 3, 3)


def _test_matrices(seed, n=64):
    """Gaussian matrices, path-average-like sums of SU(3) matrices and near-SU(3) ones."""
    rng = np.random.default_rng(seed)
    g = _gauss(rng, (n, 3, 3))
    s2 = 0.5 * (_su3(n, seed + 1) + _su3(n, seed + 2))
    near = _su3(n, seed + 3) + 0.05 * _gauss(rng, (n, 3, 3))
    return np.concatenate([g, s2, near])


# ------------------------------------------------------------------ projection
def test_projection_lands_in_su3():
    y = projection.project_sun(_test_matrices(11))
    assert np.abs(dag(y) @ y - np.eye(3)).max() < TOL
    assert np.abs(np.linalg.det(y) - 1.0).max() < TOL


def test_projection_fixes_su3_and_ignores_positive_scale():
    u = _su3(50, 21)
    assert np.abs(projection.project_sun(u) - u).max() < TOL
    a = _test_matrices(22)
    y = projection.project_sun(a)
    for c in (0.37, 5.0):
        assert np.abs(projection.project_sun(c * a) - y).max() < 1e-12


def test_projection_gauge_covariance():
    a = _test_matrices(31)
    g1 = _su3(a.shape[0], 32)
    g2 = _su3(a.shape[0], 33)
    lhs = projection.project_sun(g1 @ a @ dag(g2))
    rhs = g1 @ projection.project_sun(a) @ dag(g2)
    assert np.abs(lhs - rhs).max() < 1e-12


def test_projection_of_scaled_unitary():
    """A = c Q diag(e^{i a_j}) R with Q, R in SU(3): all singular values equal,
    so the optimal phases are equal, theta_j = -phi/3 with phi = sum a_j in
    (-pi, pi), and P(A) = A e^{-i phi/3} / c."""
    rng = np.random.default_rng(41)
    n = 40
    q, r = _su3(n, 42), _su3(n, 43)
    al = rng.uniform(-0.9, 0.9, size=(n, 3))
    x = q @ (np.exp(1j * al)[:, :, None] * np.eye(3)) @ r
    phi = al.sum(axis=1)
    y = projection.project_sun(2.5 * x)
    assert np.abs(y - x * np.exp(-1j * phi / 3.0)[:, None, None]).max() < 1e-12


def test_projection_u1_embedding():
    """diag(r e^{i psi}, r e^{-i psi}, q) with r, q > 0 projects to diag(e^{i psi}, e^{-i psi}, 1)."""
    rng = np.random.default_rng(51)
    n = 30
    r, q, ps = rng.uniform(0.2, 2, n), rng.uniform(0.2, 2, n), rng.uniform(-3, 3, n)
    a = np.zeros((n, 3, 3), dtype=np.complex128)
    a[:, 0, 0], a[:, 1, 1], a[:, 2, 2] = r * np.exp(1j * ps), r * np.exp(-1j * ps), q
    y = projection.project_sun(a)
    want = np.zeros_like(a)
    want[:, 0, 0], want[:, 1, 1], want[:, 2, 2] = np.exp(1j * ps), np.exp(-1j * ps), 1.0
    assert np.abs(y - want).max() < 1e-12


def test_projection_is_the_global_maximum():
    """Re tr(A^dag Y) against Re tr(A^dag U D V^dag) evaluated from matrices on
    a 121 x 121 grid of the two free phases (3-degree steps), against random
    SU(3) matrices, and against small perturbations of Y inside SU(3)."""
    a = _test_matrices(61, n=8)
    y = projection.project_sun(a)
    fy = np.real(np.einsum("nab,nab->n", np.conj(a), y))
    u, s, vh = np.linalg.svd(a)
    phi = np.angle(np.linalg.det(u) * np.linalg.det(vh))
    th = np.linspace(0, 2 * np.pi, 121)
    t1, t2 = np.meshgrid(th, th, indexing="ij")
    t1, t2 = t1.reshape(-1), t2.reshape(-1)
    for i in range(a.shape[0]):
        ph = np.stack([t1, t2, -phi[i] - t1 - t2], axis=1)
        cand = (u[i][None] * np.exp(1j * ph)[:, None, :]) @ vh[i][None]
        assert np.abs(np.linalg.det(cand) - 1).max() < 1e-12
        fg = np.real(np.einsum("ab,nab->n", np.conj(a[i]), cand))
        assert fg.max() <= fy[i] + 1e-12
        assert fy[i] - fg.max() < 2e-3 * s[i].sum()
    z = _su3(4000, 62)
    for i in range(a.shape[0]):
        assert projection.distance2(a[i], y[i]) <= projection.distance2(a[i][None], z).min() + 1e-12
        assert projection.distance2(a[i], y[i]) <= projection.distance2(a[i], projection.naive_sun(a[i])) + 1e-12
    # local optimality: Y exp(i eps H) for traceless Hermitian H is farther from A
    rng = np.random.default_rng(63)
    for _ in range(20):
        h = _gauss(rng, (3, 3))
        h = 0.5 * (h + dag(h))
        h -= np.trace(h) / 3 * np.eye(3)
        w, v = np.linalg.eigh(h)
        e = (v * np.exp(1e-3j * w)) @ dag(v)
        d0 = projection.distance2(a, y)
        assert np.all(projection.distance2(a, y @ e) >= d0 - 1e-14)


def test_projection_lagrange_condition():
    """At the constrained maximum s_j sin(theta_j) is the same for all j."""
    a = _test_matrices(71)
    u, s, vh = np.linalg.svd(a)
    phi = np.angle(np.linalg.det(u) * np.linalg.det(vh))
    th = projection.maximise_phases(s, phi)
    m = s * np.sin(th)
    assert np.abs(m - m[:, :1]).max() < 1e-12


def test_projection_footnote_negative_determinant():
    """det(U + V) is real for U, V in SU(3) (the paper's footnote in Sec. 5.2);
    with V = diag(e^{ib}, e^{ib}, e^{-2ib}), b = 2, det(1 + V) < 0, where the
    cube-root recipe sits on its branch cut.  The projection still returns an
    SU(3) matrix at least as close as the cube-root one and as any of many
    random SU(3) matrices."""
    b = 2.0
    a = np.eye(3, dtype=np.complex128) + np.diag([np.exp(1j * b), np.exp(1j * b), np.exp(-2j * b)])
    d = np.linalg.det(a)
    assert abs(d.imag) < 1e-14 and d.real < 0
    g1, g2 = _su3(1, 81)[0], _su3(1, 82)[0]
    a = g1 @ a @ dag(g2)
    y = projection.project_sun(a)
    assert np.abs(dag(y) @ y - np.eye(3)).max() < TOL and abs(np.linalg.det(y) - 1) < TOL
    assert projection.distance2(a, y) <= projection.distance2(a, projection.naive_sun(a)) + 1e-12
    assert projection.distance2(a, y) <= projection.distance2(a[None], _su3(4000, 83)).min() + 1e-12


def test_project_un_two_forms():
    """Eq. def_projection: A (A^dag A)^{-1/2} = (A A^dag)^{-1/2} A, via eigh."""
    a = _test_matrices(91)

    def inv_sqrt(h):
        w, v = np.linalg.eigh(h)
        return (v / np.sqrt(w)[:, None, :]) @ dag(v)

    x = projection.project_un(a)
    assert np.abs(x - a @ inv_sqrt(dag(a) @ a)).max() < 1e-11
    assert np.abs(x - inv_sqrt(a @ dag(a)) @ a).max() < 1e-11


# ------------------------------------------------------------------ U(1) embedding helpers
def _u1_links(dims, seed, amp=1.0):
    """Links diag(e^{i b}, e^{-i b}, 1) with random phases b[mu, t, z, y, x]."""
    rng = np.random.default_rng(seed)
    beta = rng.uniform(-amp, amp, size=(4,) + synth.lattice_shape(dims))
    u = np.zeros(beta.shape + (3, 3), dtype=np.complex128)
    u[..., 0, 0], u[..., 1, 1], u[..., 2, 2] = np.exp(1j * beta), np.exp(-1j * beta), 1.0
    return beta, u


def _sh(f, d):
    """f(x + d) for a scalar field indexed [t, z, y, x]."""
    for mu in range(4):
        if d[mu]:
            f = np.roll(f, -d[mu], axis=3 - mu)
    return f


def _e(mu, s=1):
    e = [0, 0, 0, 0]
    e[mu] = s
    return e


def _plus(*vs):
    return [sum(v[i] for v in vs) for i in range(4)]


# ------------------------------------------------------------------ APE
def test_ape_alpha_zero_and_pure_gauge():
    dims = (4, 3, 3, 4)
    u = synth.gauge_links(dims, 0.4, 101)
    assert np.abs(smearing.ape(u, 0.0) - u).max() < TOL
    g = synth.random_su3_field(dims, 102)
    pure = synth.gauge_transform_links(synth.unit_links(dims), g)
    assert np.abs(smearing.ape(pure, smearing.ALPHA_PAPER) - pure).max() < 1e-12


def test_ape_gauge_covariance():
    dims = (3, 4, 3, 3)
    u = synth.gauge_links(dims, 0.5, 111)
    g = synth.random_su3_field(dims, 112)
    lhs = smearing.ape(synth.gauge_transform_links(u, g), 0.72)
    rhs = synth.gauge_transform_links(smearing.ape(u, 0.72), g)
    assert np.abs(lhs - rhs).max() < 1e-12


def test_ape_u1_closed_form():
    """For links diag(e^{ib}, e^{-ib}, 1) every loop is diag(e^{i Phi}, e^{-i Phi}, 1)
    with Phi the sum of signed link phases around it, so the projected argument
    is diag(z/|z|, conj(z)/|z|, 1), z = 1 - alpha + alpha/6 sum e^{i Phi}."""
    dims = (4, 3, 4, 3)
    alpha = 0.72
    beta, u = _u1_links(dims, 121)
    v = smearing.ape(u, alpha)
    for mu in range(4):
        z = np.full(beta.shape[1:], 1.0 - alpha, dtype=np.complex128)
        for nu in range(4):
            if nu == mu:
                continue
            bm, bn = beta[mu], beta[nu]
            ph_p = bn + _sh(bm, _e(nu)) - _sh(bn, _e(mu)) - bm
            ph_m = -_sh(bn, _e(nu, -1)) + _sh(bm, _e(nu, -1)) + _sh(bn, _plus(_e(nu, -1), _e(mu))) - bm
            z += alpha / 6.0 * (np.exp(1j * ph_p) + np.exp(1j * ph_m))
        ang = beta[mu] + np.angle(z)
        assert np.abs(v[mu][..., 0, 0] - np.exp(1j * ang)).max() < 1e-12
        assert np.abs(v[mu][..., 1, 1] - np.exp(-1j * ang)).max() < 1e-12
        assert np.abs(v[mu][..., 2, 2] - 1.0).max() < 1e-12
        off = v[mu].copy()
        for k in range(3):
            off[..., k, k] = 0
        assert np.abs(off).max() < 1e-12


def test_ape_sampled_sites_match_whole_lattice():
    from oracle.transporters import make_site_getter
    dims = (4, 3, 3, 4)
    u = synth.gauge_links(dims, 0.4, 131)
    v = smearing.ape(u, 0.72)
    sites = np.array([[0, 0, 0, 0], [3, 2, 1, 3], [1, 1, 2, 0]])
    get = make_site_getter(sites, dims)
    for mu in range(4):
        vs = smearing.ape_link(u, mu, 0.72, get)
        for j, (x, y, z, t) in enumerate(sites):
            assert np.abs(vs[j] - v[mu][t, z, y, x]).max() < 1e-14


# ------------------------------------------------------------------ clover
def test_sigma_algebra():
    g = gammas()
    g5 = gamma5()
    for mu in range(4):
        for nu in range(4):
            s = clover.sigma(mu, nu)
            assert np.abs(s - dag(s)).max() < TOL
            assert np.abs(s @ g5 - g5 @ s).max() < TOL
            if mu != nu:
                assert np.abs(s - 1j * g[mu] @ g[nu]).max() < TOL
            else:
                assert np.abs(s).max() == 0


def test_clover_vanishes_for_unit_and_pure_gauge_links():
    dims = (3, 3, 4, 3)
    assert np.abs(clover.clover_matrix(synth.unit_links(dims))).max() == 0
    pure = synth.gauge_transform_links(synth.unit_links(dims), synth.random_su3_field(dims, 141))
    assert np.abs(clover.clover_matrix(pure)).max() < 1e-13


def test_field_strength_hermitian_traceless_covariant():
    dims = (3, 4, 3, 3)
    u = synth.gauge_links(dims, 0.5, 151)
    g = synth.random_su3_field(dims, 152)
    ug = synth.gauge_transform_links(u, g)
    for mu, nu in itertools.combinations(range(4), 2):
        f = clover.field_strength(u, mu, nu)
        assert np.abs(f - dag(f)).max() < TOL
        assert np.abs(np.trace(f, axis1=-2, axis2=-1)).max() < TOL
        assert np.abs(clover.field_strength(ug, mu, nu) - g @ f @ dag(g)).max() < 1e-13
        assert np.abs(clover.field_strength(u, nu, mu) + f).max() < TOL
    c = clover.clover_matrix(u)
    assert np.abs(c - dag(c)).max() < TOL
    g5 = np.kron(gamma5(), np.eye(3))
    assert np.abs(c @ g5 - g5 @ c).max() < TOL


def test_field_strength_u1_closed_form():
    """Links diag(e^{ib}, e^{-ib}, 1): F_{mu nu} = diag(f, -f, 0) with
    f = (1/4) sum over the four leaves of sin(Phi_leaf)."""
    dims = (3, 4, 3, 4)
    beta, u = _u1_links(dims, 161)
    for mu, nu in itertools.combinations(range(4), 2):
        bm, bn = beta[mu], beta[nu]
        pm, pn, mm, mn = _e(mu), _e(nu), _e(mu, -1), _e(nu, -1)
        p1 = bm + _sh(bn, pm) - _sh(bm, pn) - bn
        p2 = bn - _sh(bm, _plus(mm, pn)) - _sh(bn, mm) + _sh(bm, mm)
        p3 = -_sh(bm, mm) - _sh(bn, _plus(mm, mn)) + _sh(bm, _plus(mm, mn)) + _sh(bn, mn)
        p4 = -_sh(bn, mn) + _sh(bm, mn) + _sh(bn, _plus(mn, pm)) - bm
        f = 0.25 * (np.sin(p1) + np.sin(p2) + np.sin(p3) + np.sin(p4))
        fs = clover.field_strength(u, mu, nu)
        assert np.abs(fs[..., 0, 0] - f).max() < 1e-14
        assert np.abs(fs[..., 1, 1] + f).max() < 1e-14
        assert np.abs(fs[..., 2, 2]).max() < 1e-14


def test_clover_weak_constant_field_matches_continuum_form():
    """A constant abelian field in the (x, y) plane with plaquette angle B
    (quantised: B = 2 pi / (Lx Ly)) has f = sin(B) everywhere, and the clover
    term is -(1/2) sigma_xy (x) diag(f, -f, 0)."""
    dims = (4, 4, 2, 2)
    lx, ly = dims[0], dims[1]
    b = 2 * np.pi / (lx * ly)
    shp = synth.lattice_shape(dims)
    t, z, y, x = np.meshgrid(*[np.arange(n) for n in shp], indexing="ij")
    beta = np.zeros((4,) + shp)
    beta[1] = b * x                                  # U_y(x) = e^{i B x}
    beta[0] = np.where(x == lx - 1, -b * lx * y, 0.0)  # twist closes the torus
    u = np.zeros(beta.shape + (3, 3), dtype=np.complex128)
    u[..., 0, 0], u[..., 1, 1], u[..., 2, 2] = np.exp(1j * beta), np.exp(-1j * beta), 1.0
    f = clover.field_strength(u, 0, 1)
    assert np.abs(f[..., 0, 0] - np.sin(b)).max() < 1e-13
    want = -0.5 * np.kron(clover.sigma(0, 1), np.diag([np.sin(b), -np.sin(b), 0.0]))
    assert np.abs(clover.clover_matrix(u) - want).max() < 1e-13


# ------------------------------------------------------------------ production operator
def test_projected_transporters_u1_closed_form():
    """For diag(e^{ib}, e^{-ib}, 1) links the path average is diag(a, conj(a), 1)
    with a the average of e^{i (sum of signed phases along the path)}, and the
    projection gives diag(a/|a|, conj(a)/|a|, 1)."""
    dims = (3, 3, 4, 3)
    beta, u = _u1_links(dims, 171)
    for n in [(1, -1, 0, 0), (0, 1, 1, -1), (-1, 1, -1, 1), (1, 0, 0, 0)]:
        supp = [mu for mu in range(4) if n[mu]]
        acc = 0
        for order in itertools.permutations(supp):
            d = [0, 0, 0, 0]
            ph = 0
            for mu in order:
                if n[mu] > 0:
                    ph = ph + _sh(beta[mu], d)
                else:
                    ph = ph - _sh(beta[mu], _plus(d, _e(mu, -1)))
                d[mu] += n[mu]
            acc = acc + np.exp(1j * ph)
        a = acc / len(list(itertools.permutations(supp)))
        w = production.transporter_su3(u, n)
        assert np.abs(w[..., 0, 0] - a / np.abs(a)).max() < 1e-12
        assert np.abs(w[..., 1, 1] - np.conj(a) / np.abs(a)).max() < 1e-12
        assert np.abs(w[..., 2, 2] - 1).max() < 1e-12


def test_production_free_limit_equals_plain_operator():
    dims = (3, 3, 3, 4)
    u = synth.unit_links(dims)
    psi = synth.gaussian_spinor(dims, 181)
    assert np.abs(production.apply(u, psi, 0.1) - dirac.apply(u, psi, 0.1)).max() < 1e-13


def test_production_gamma5_hermiticity_and_adjoint():
    dims = (3, 3, 3, 3)
    u = smearing.ape(synth.gauge_links(dims, 0.4, 191), 0.72)
    psi = synth.gaussian_spinor(dims, 192)
    chi = synth.gaussian_spinor(dims, 193)
    g5 = gamma5()
    sand = np.einsum("st,...tc->...sc", g5, production.apply(u, np.einsum("st,...tc->...sc", g5, psi), 0.1))
    dg = production.apply_dag(u, psi, 0.1)
    assert np.abs(dg - sand).max() < 1e-13 * np.abs(dg).max()
    lhs = np.vdot(chi, production.apply(u, psi, 0.1))
    rhs = np.vdot(production.apply_dag(u, chi, 0.1), psi)
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)


def test_production_gauge_covariance():
    dims = (3, 3, 3, 3)
    u = synth.gauge_links(dims, 0.4, 201)
    g = synth.random_su3_field(dims, 202)
    psi = synth.gaussian_spinor(dims, 203)
    lhs = production.apply(synth.gauge_transform_links(u, g), synth.gauge_transform_spinor(psi, g), 0.1)
    rhs = synth.gauge_transform_spinor(production.apply(u, psi, 0.1), g)
    assert np.abs(lhs - rhs).max() < 1e-12


def test_production_sampled_sites_match():
    dims = (3, 4, 3, 3)
    u = synth.gauge_links(dims, 0.4, 211)
    psi = synth.gaussian_spinor(dims, 212)
    full = production.apply(u, psi, 0.1)
    sites = np.array([[0, 0, 0, 0], [2, 3, 1, 2], [1, 2, 2, 0]])
    part = production.apply_at(u, psi, 0.1, sites)
    for j, (x, y, z, t) in enumerate(sites):
        assert np.abs(part[j] - full[t, z, y, x]).max() < 1e-14


def test_production_clover_only_adds_the_local_term():
    dims = (3, 3, 3, 3)
    u = synth.gauge_links(dims, 0.4, 221)
    psi = synth.gaussian_spinor(dims, 222)
    diff = production.apply(u, psi, 0.1, csw=1.0) - production.apply(u, psi, 0.1, csw=0.0)
    assert np.abs(diff - clover.apply_clover(u, psi, 1.0)).max() < 1e-13
