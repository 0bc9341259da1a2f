"""GPU overlap operator (Sec. 7) against the dense, exact oracle: Lanczos
Ritz values against the eigenvalues of D^dag D, sign(H) and D_ov,m against
the exact sign function to the Chebyshev interpolant's error bound, the
deflated form with given orthonormal vectors, and, at 16^3 x 32 where no
dense oracle exists, the identities sign(H)^2 = 1 and Ginsparg-Wilson.

Tolerances: the GPU reports e = max over [lo, hi] of |1 - sqrt(x) p(x)|;
sign(H) psi then differs from the exact value by at most e |psi| (per
eigencomponent), so the bound is e + 1e-12 relative (FP64 rounding of
~2 degree applications)."""
import numpy as np
import pytest

import synth
from oracle import overlap as oov
from tests.helpers import dev, log, soa_to_canon

pytestmark = pytest.mark.gpu

DIMS = (4, 2, 2, 4)
RHO = 1.0


@pytest.fixture(scope="module")
def bri():
    import paper_1012_3615_amd as m
    return m


@pytest.fixture(scope="module")
def setup(bri):
    u = synth.gauge_links(DIMS, 0.5, 8201)
    dk = oov.kernel_matrix(u, RHO)
    ev = oov.ritz_reference(dk)
    U = bri.bri_pack_links(DIMS, dev(u), bri.F64)
    op = bri.Operator(bri.bri_build_transporters(DIMS, U, bri.F64, 80))
    return u, dk, ev, op


def _flat(x):
    return x.reshape(x.shape[0], -1)


def _degree(lo, hi, target):
    """Smallest degree in a doubling ladder whose interpolant meets the target."""
    for deg in (50, 100, 200, 400, 800, 1600, 3200):
        if oov.inv_sqrt_chebyshev(lo, hi, deg)[1] < target:
            return deg
    raise AssertionError("spectral interval too wide")


def test_lanczos_ritz_values(bri, setup):
    _, _, ev, op = setup
    log("lanczos ritz 4x2x2x4")
    v0 = bri.bri_pack_spinor(DIMS, dev(synth.gaussian_spinor(DIMS, 8202, nrhs=1)), bri.F64)
    # full re-orthogonalisation: all 768 eigenvalues are resolved after 768 steps
    a, b, basis = bri.bri_lanczos(DIMS, op, -RHO, 768, v0, keep_basis=True)
    r = bri.bri_ritz_values(a, b, filter=False)
    assert len(r) == 768
    assert np.abs(r - ev).max() < 1e-10 * ev.max()
    # the kept basis is orthonormal
    q = _flat(soa_to_canon(DIMS, basis[:64]).reshape(64, -1))
    assert np.abs(q.conj() @ q.T - np.eye(64)).max() < 1e-12
    # three-term recurrence only, 200 steps, spurious copies filtered: the
    # extremes converge, and every kept value lies inside the spectrum
    a, b, _ = bri.bri_lanczos(DIMS, op, -RHO, 200, v0)
    r = bri.bri_ritz_values(a, b, filter=True)
    assert abs(r[-1] - ev[-1]) < 1e-10 * ev[-1]
    assert abs(r[0] - ev[0]) < 1e-8 * ev[-1]
    assert r[0] >= ev[0] - 1e-10 and r[-1] <= ev[-1] * (1 + 1e-12)


@pytest.mark.parametrize("degree", [60, 160])
def test_sign_matches_exact(bri, setup, degree):
    u, dk, ev, op = setup
    log(f"sign(H) degree {degree}")
    lo, hi = 0.95 * ev[0], 1.05 * ev[-1]
    psi = synth.gaussian_spinor(DIMS, 8203, nrhs=2)
    x = bri.bri_pack_spinor(DIMS, dev(psi), bri.F64)
    out, err = bri.bri_sign_h(DIMS, op, -RHO, x, lo, hi, degree)
    c, err_o = oov.inv_sqrt_chebyshev(lo, hi, degree)
    assert abs(err - err_o) <= 1e-6 * err_o + 1e-15
    s = oov.sign_matrix(oov.hermitian_kernel(dk))
    got = _flat(soa_to_canon(DIMS, out))
    want = (s @ _flat(psi).T).T
    for r in range(2):
        assert np.linalg.norm(got[r] - want[r]) <= (err + 1e-12) * np.linalg.norm(psi[r])


def test_overlap_apply_matches_exact(bri, setup):
    u, dk, ev, op = setup
    lo, hi = 0.95 * ev[0], 1.05 * ev[-1]
    psi = synth.gaussian_spinor(DIMS, 8204, nrhs=3)
    x = bri.bri_pack_spinor(DIMS, dev(psi), bri.F64)
    deg = _degree(lo, hi, 1e-11)
    for m in (0.0, 0.05):
        log(f"overlap apply m={m} degree {deg}")
        out, err = bri.bri_overlap_apply(DIMS, op, x, RHO, m, lo, hi, deg)
        assert err < 1e-11
        want = (oov.overlap_matrix(dk, RHO, m) @ _flat(psi).T).T
        got = _flat(soa_to_canon(DIMS, out))
        for r in range(3):
            assert np.linalg.norm(got[r] - want[r]) <= (2 * err + 1e-12) * np.linalg.norm(psi[r])


def test_sign_with_deflation(bri, setup):
    """Given orthonormal vectors v_i and signs s_i (seeded, not eigenvectors),
    the library computes sum_i s_i v_i <v_i, psi> + sign(H)(psi - sum_i v_i <v_i, psi>);
    the oracle forms the same with the exact sign."""
    u, dk, ev, op = setup
    log("sign(H) deflated")
    n = 12 * synth.volume(DIMS)
    rng = np.random.default_rng(8205)
    q, _ = np.linalg.qr(rng.standard_normal((n, 5)) + 1j * rng.standard_normal((n, 5)))
    sg = np.array([0.7, -1.3, 2.0, -0.1, 0.4])
    vecs = q.T.reshape((5,) + synth.lattice_shape(DIMS) + (4, 3))
    V = bri.bri_pack_spinor(DIMS, dev(vecs), bri.F64)
    psi = synth.gaussian_spinor(DIMS, 8206, nrhs=2)
    x = bri.bri_pack_spinor(DIMS, dev(psi), bri.F64)
    lo, hi = 0.95 * ev[0], 1.05 * ev[-1]
    out, err = bri.bri_sign_h(DIMS, op, -RHO, x, lo, hi, _degree(lo, hi, 1e-11), low_vecs=V, low_evals=sg)
    s = oov.sign_matrix(oov.hermitian_kernel(dk))
    got = _flat(soa_to_canon(DIMS, out))
    for r in range(2):
        p = _flat(psi)[r]
        c = q.conj().T @ p
        want = q @ (np.sign(sg) * c) + s @ (p - q @ c)
        assert np.linalg.norm(got[r] - want) <= (err + 1e-12) * np.linalg.norm(p)


def test_overlap_identities_16_32(bri):
    """16^3 x 32, links eps = 0.3: spectral bounds of D^dag D from Lanczos
    (three-term recurrence, filtered; the interval widened by 10% below and
    5% above), then sign(H)^2 psi = psi and the Ginsparg-Wilson relation
    gamma5 D_ov + D_ov gamma5 = D_ov gamma5 D_ov / rho on a random field."""
    import torch
    dims = (16, 16, 16, 32)
    log("overlap identities 16^3x32")
    u = synth.gauge_links(dims, 0.3, 8301)
    U = bri.bri_pack_links(dims, dev(u), bri.F64)
    op = bri.Operator(bri.bri_build_transporters(dims, U, bri.F64, 80))
    v0 = bri.bri_pack_spinor(dims, dev(synth.gaussian_spinor(dims, 8302, nrhs=1)), bri.F64)
    a, b, _ = bri.bri_lanczos(dims, op, -RHO, 300, v0)
    r = bri.bri_ritz_values(a, b)
    lo, hi = 0.9 * r[0], 1.05 * r[-1]
    x = bri.bri_pack_spinor(dims, dev(synth.gaussian_spinor(dims, 8303, nrhs=1)), bri.F64)
    deg = _degree(lo, hi, 1e-10)
    s1, err = bri.bri_sign_h(dims, op, -RHO, x, lo, hi, deg)
    s2, _ = bri.bri_sign_h(dims, op, -RHO, s1, lo, hi, deg)
    log(f"ritz [{r[0]:.4g}, {r[-1]:.4g}] degree {deg} err {err:.3g}")
    assert err < 1e-10
    assert float(torch.linalg.norm(s2 - x) / torch.linalg.norm(x)) <= 3 * err + 1e-11
    # Ginsparg-Wilson on the output: (g5 D + D g5 - D g5 D / rho) x = 0
    def ov(y):
        return bri.bri_overlap_apply(dims, op, y, RHO, 0.0, lo, hi, deg)[0]

    def g5(y):
        z = y.clone()
        z[:, 6:] *= -1
        return z

    dx = ov(x)
    lhs = g5(dx) + ov(g5(x))
    rhs = ov(g5(dx)) / RHO
    assert float(torch.linalg.norm(lhs - rhs) / torch.linalg.norm(x)) <= 20 * err + 1e-10


def test_lowmodes_and_deflated_sign(bri, setup):
    """The 6 modes of H of smallest |eigenvalue| from 300 re-orthogonalised
    Lanczos steps and Rayleigh-Ritz: eigenvalues against the oracle's dense
    eigh, orthonormal, eigenvectors of the oracle's H; deflating them lets a
    polynomial on the reduced interval [0.95 lambda_7^2, 1.05 lambda_max^2]
    reach the exact sign, which the same polynomial without deflation misses."""
    u, dk, ev, op = setup
    log("low modes 4x2x2x4")
    h = oov.hermitian_kernel(dk)
    lam = np.linalg.eigvalsh(h)
    lam = lam[np.argsort(np.abs(lam))]
    n_low = 6
    v0 = bri.bri_pack_spinor(DIMS, dev(synth.gaussian_spinor(DIMS, 8207, nrhs=1)), bri.F64)
    V, mu, res = bri.bri_overlap_lowmodes(DIMS, op, -RHO, 300, v0, n_low)
    assert np.abs(mu - lam[:n_low]).max() < 1e-9 * np.abs(lam).max()
    assert res.max() < 1e-8
    q = _flat(soa_to_canon(DIMS, V))
    assert np.abs(q.conj() @ q.T - np.eye(n_low)).max() < 1e-10
    for i in range(n_low):
        assert np.linalg.norm(h @ q[i] - mu[i] * q[i]) < 1e-8
    lo, hi = 0.95 * lam[n_low] ** 2, 1.05 * ev[-1]
    deg = _degree(lo, hi, 1e-11)
    psi = synth.gaussian_spinor(DIMS, 8208, nrhs=1)
    x = bri.bri_pack_spinor(DIMS, dev(psi), bri.F64)
    s = oov.sign_matrix(h)
    want = s @ _flat(psi)[0]
    out, err = bri.bri_sign_h(DIMS, op, -RHO, x, lo, hi, deg, low_vecs=V, low_evals=mu)
    got = _flat(soa_to_canon(DIMS, out))[0]
    assert np.linalg.norm(got - want) <= (err + 1e-8) * np.linalg.norm(want)
    out0, _ = bri.bri_sign_h(DIMS, op, -RHO, x, lo, hi, deg)
    got0 = _flat(soa_to_canon(DIMS, out0))[0]
    assert np.linalg.norm(got0 - want) > 1e3 * np.linalg.norm(got - want)


@pytest.mark.parametrize("rho,m", [(0.7, 0.0), (1.6, 0.1)])
def test_overlap_other_rho(bri, setup, rho, m):
    """D_ov,m at rho = 0.7 and 1.6 (kernel at mass -rho) against the dense exact
    operator, degree chosen from the Ritz interval of that kernel."""
    u, _, _, op = setup
    log(f"overlap rho={rho} m={m}")
    dk = oov.kernel_matrix(u, rho)
    ev = oov.ritz_reference(dk)
    lo, hi = 0.95 * ev[0], 1.05 * ev[-1]
    deg = _degree(lo, hi, 1e-11)
    psi = synth.gaussian_spinor(DIMS, 8209, nrhs=2)
    x = bri.bri_pack_spinor(DIMS, dev(psi), bri.F64)
    out, err = bri.bri_overlap_apply(DIMS, op, x, rho, m, lo, hi, deg)
    want = (oov.overlap_matrix(dk, rho, m) @ _flat(psi).T).T
    got = _flat(soa_to_canon(DIMS, out))
    for r in range(2):
        assert np.linalg.norm(got[r] - want[r]) <= (2 * rho * err + 1e-12) * np.linalg.norm(psi[r])
