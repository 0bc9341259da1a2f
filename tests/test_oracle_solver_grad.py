"""Pins for the oracle's solver and gradients (no GPU)."""
import math

import numpy as np
import pytest

import synth
from oracle import dirac, free, grad, solver


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_cgne_matches_dense_solve():
    dims = (2, 2, 2, 4)
    u = synth.gauge_links(dims, 0.3, seed=31)
    b = synth.gaussian_spinor(dims, seed=32)
    x, it, res = solver.cgne(u, b, 0.1, tol=1e-12)
    assert res <= 1e-12
    d = dirac.dense_matrix(u, 0.1)
    xd = np.linalg.solve(d, b.reshape(-1)).reshape(b.shape)
    assert rel(x, xd) < 1e-9
    assert it > 5


def test_fft_propagator_matches_cgne_free_field():
    dims = (4, 4, 4, 4)
    u = synth.unit_links(dims)
    b = synth.point_sources(dims)[5]
    xf = free.propagator_solve(dims, b, 0.2)
    x, _, res = solver.cgne(u, b, 0.2, tol=1e-11)
    assert res <= 1e-11
    assert rel(x, xf) < 1e-9
    assert rel(dirac.apply(u, xf, 0.2), b) < 1e-12


DIMS_G = (2, 3, 2, 2)
MASS = 0.1


@pytest.fixture(scope="module")
def grad_setup():
    u = synth.gauge_links(DIMS_G, 0.4, seed=41)
    chi = synth.gaussian_spinor(DIMS_G, seed=42)
    psi = synth.gaussian_spinor(DIMS_G, seed=43)
    return u, chi, psi


def _fd(f, h=1e-5):
    return (f(h) - f(-h)) / (2 * h)


def test_psi_gradient_central_difference(grad_setup):
    u, chi, psi = grad_setup
    g = grad.grad_psi(u, chi, MASS)
    rng = np.random.default_rng(44)
    for _ in range(6):
        idx = tuple(int(rng.integers(s)) for s in psi.shape)
        for unit, part in ((1.0, "re"), (1j, "im")):
            def s_of(h):
                p = psi.copy()
                p[idx] += unit * h
                return grad.action(u, chi, p, MASS)
            fd = _fd(s_of)
            an = g[idx].real if part == "re" else g[idx].imag
            assert abs(fd - an) <= 1e-7 * max(1.0, abs(an))


def test_link_gradient_central_difference(grad_setup):
    u, chi, psi = grad_setup
    g = grad.grad_links(u, chi, psi, MASS)
    gmax = np.abs(g).max()
    rng = np.random.default_rng(45)
    for _ in range(10):
        idx = tuple(int(rng.integers(s)) for s in u.shape)
        for unit, part in ((1.0, "re"), (1j, "im")):
            def s_of(h):
                uu = u.copy()
                uu[idx] += unit * h
                return grad.action(uu, chi, psi, MASS)
            fd = _fd(s_of)
            an = g[idx].real if part == "re" else g[idx].imag
            assert abs(fd - an) <= 1e-6 * gmax, (idx, part, fd, an)


def test_link_gradient_linear_in_chi_and_psi(grad_setup):
    u, chi, psi = grad_setup
    g1 = grad.grad_links(u, chi, psi, MASS)
    g2 = grad.grad_links(u, 2.0 * chi, psi, MASS)
    assert rel(g2, 2.0 * g1) < 1e-14
    # S is real-linear in chi: i*chi gives S' = Re<i chi, D psi> = Im<chi, D psi>
    s_re = grad.action(u, chi, psi, MASS)
    assert math.isfinite(s_re)


def test_link_gradient_generic_table_central_difference(grad_setup):
    """The same chain rule with the hypercube column of Tab. rholambda."""
    from oracle import ultralocal
    u, chi, psi = grad_setup
    tab = ultralocal.HYPERCUBE
    g = grad.grad_links(u, chi, psi, MASS, table=tab)
    assert rel(g, grad.grad_links(u, chi, psi, MASS)) > 1e-3  # the table matters
    gmax = np.abs(g).max()
    rng = np.random.default_rng(46)
    for _ in range(8):
        idx = tuple(int(rng.integers(s)) for s in u.shape)
        for unit, part in ((1.0, "re"), (1j, "im")):
            def s_of(h):
                uu = u.copy()
                uu[idx] += unit * h
                return grad.action(uu, chi, psi, MASS, table=tab)
            fd = _fd(s_of)
            an = g[idx].real if part == "re" else g[idx].imag
            assert abs(fd - an) <= 1e-6 * gmax, (idx, part, fd, an)
    gp = grad.grad_psi(u, chi, MASS, table=tab)
    idx = (1, 0, 2, 1, 3, 2)
    def s_psi(h):
        p = psi.copy()
        p[idx] += h
        return grad.action(u, chi, p, MASS, table=tab)
    assert abs(_fd(s_psi) - gp[idx].real) <= 1e-7 * max(1.0, abs(gp[idx].real))
