"""Pins of the overlap oracle (Sec. 7, Eqs. def_over, def_mass): the
algebraic identities every exact overlap operator satisfies, and the free
field from the momentum-space symbol."""
import numpy as np
import pytest

import synth
from oracle import dirac, free, overlap
from oracle.gamma import gamma5, gammas

TOL = 1e-12


@pytest.fixture(scope="module", params=[(2, 2, 2, 2), (3, 2, 2, 3)])
def gauged(request):
    dims = request.param
    u = synth.gauge_links(dims, 0.5, 8001)
    dk = overlap.kernel_matrix(u, 1.0)
    return dims, u, dk


def test_sign_squares_to_one(gauged):
    _, _, dk = gauged
    s = overlap.sign_matrix(overlap.hermitian_kernel(dk))
    assert np.abs(s @ s - np.eye(s.shape[0])).max() < TOL
    assert np.abs(s - s.conj().T).max() < TOL


@pytest.mark.parametrize("rho", [1.0, 0.7, 1.6])
def test_ginsparg_wilson_and_circle(gauged, rho):
    dims, u, _ = gauged
    dk = overlap.kernel_matrix(u, rho)
    d = overlap.overlap_matrix(dk, rho)
    g5 = overlap.gamma5_full(d.shape[0] // 12)
    assert np.abs(g5 @ d + d @ g5 - d @ g5 @ d / rho).max() < 1e-11
    z = np.linalg.eigvals(d)
    assert np.abs(np.abs(z - rho) - rho).max() < 1e-11
    assert np.abs(g5 @ d @ g5 - d.conj().T).max() < TOL


def test_massive_overlap_circle(gauged):
    _, _, dk = gauged
    rho, m = 1.0, 0.08
    d = overlap.overlap_matrix(dk, rho, mass=m)
    z = np.linalg.eigvals(d)
    assert np.abs(np.abs(z - (rho + m / 2)) - (rho - m / 2)).max() < 1e-11


def test_free_field_closed_form():
    """Unit links: D_ov(k) = rho [1 + (Dhat(k) - rho) / sqrt((A(k) - rho)^2 + |s(k)|^2)],
    checked on plane waves e^{ikx} chi against the dense operator, and the
    4x4 form against gamma5 sign(gamma5 (Dhat - rho)) from a 4x4 eigh."""
    dims, rho = (4, 2, 2, 4), 1.0
    u = synth.unit_links(dims)
    d = overlap.overlap_matrix(overlap.kernel_matrix(u, rho), rho)
    g5 = gamma5()
    rng = np.random.default_rng(8101)
    for mom in [(0, 0, 0, 0), (1, 0, 1, 2), (2, 1, 0, 3), (3, 1, 1, 1)]:
        k = np.array([2 * np.pi * mom[mu] / dims[mu] for mu in range(4)])
        dh = free.symbol(k, 0.0)
        a, s = free.a_of_k(k, 0.0), free.s_of_k(k)
        closed = rho * (np.eye(4) + (dh - rho * np.eye(4)) / np.sqrt((a - rho) ** 2 + np.dot(s, s)))
        h = g5 @ (dh - rho * np.eye(4))
        w, v = np.linalg.eigh(h)
        via_sign = rho * (np.eye(4) + g5 @ (v * np.sign(w)) @ v.conj().T)
        assert np.abs(closed - via_sign).max() < 1e-13
        chi = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        pw = synth.plane_wave(dims, mom, chi)
        out = (d @ pw.reshape(-1)).reshape(pw.shape)
        want = synth.plane_wave(dims, mom, closed @ chi)
        assert np.abs(out - want).max() < 1e-12


def test_chebyshev_interpolant():
    lo, hi = 0.05, 3.0
    c, err = overlap.inv_sqrt_chebyshev(lo, hi, 40)
    ref = np.polynomial.chebyshev.chebinterpolate(
        lambda t: 1.0 / np.sqrt(0.5 * (hi - lo) * t + 0.5 * (hi + lo)), 40)
    assert np.abs(c - ref).max() < 1e-12
    errs = [overlap.inv_sqrt_chebyshev(lo, hi, n)[1] for n in (10, 20, 40, 80)]
    assert all(errs[i + 1] < errs[i] for i in range(3)) and errs[-1] < 1e-8


def test_ritz_reference_matches_normal_operator(gauged):
    _, _, dk = gauged
    h = overlap.hermitian_kernel(dk)
    ev = overlap.ritz_reference(dk)
    assert np.allclose(np.sort(np.linalg.eigvalsh(h) ** 2), ev, atol=1e-12)
    assert ev[0] >= -1e-12
