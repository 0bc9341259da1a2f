"""Pins for the oracle's gamma matrices, transporters and Dirac operator (no GPU)."""
import itertools

import numpy as np
import pytest

import synth
from oracle import dirac, factorized, free, gamma, transporters
from oracle.lattice import all_offsets, dag, hops, shift


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


# ---------------------------------------------------------------- gamma basis

def test_gamma_clifford_and_hermitian():
    g = gamma.gammas()
    for mu in range(4):
        assert np.allclose(g[mu], dag(g[mu]))
        for nu in range(4):
            assert np.allclose(g[mu] @ g[nu] + g[nu] @ g[mu], 2 * (mu == nu) * np.eye(4))
    g5 = gamma.gamma5()
    assert np.allclose(g5, np.diag([1, 1, -1, -1]))
    for mu in range(4):
        assert np.allclose(g5 @ g[mu], -g[mu] @ g5)


# ---------------------------------------------------------------- transporters

DIMS_SMALL = (3, 3, 3, 3)


@pytest.fixture(scope="module")
def links_small():
    return synth.gauge_links(DIMS_SMALL, 0.5, seed=11)


def test_path_counts():
    counts = {k: set() for k in range(1, 5)}
    for n in all_offsets():
        counts[hops(n)].add(len(transporters.path_orderings(n)))
    assert counts == {1: {1}, 2: {2}, 3: {6}, 4: {24}}


def test_unit_links_give_identity_transporters():
    u = synth.unit_links((2, 3, 2, 3))
    for n in all_offsets():
        w = transporters.transporter(u, n)
        assert np.allclose(w, np.eye(3), atol=1e-15)


def test_two_hop_closed_form(links_small):
    for mu, nu in itertools.combinations(range(4), 2):
        n = [0, 0, 0, 0]
        n[mu] = n[nu] = 1
        w = transporters.transporter(links_small, tuple(n))
        assert rel(w, transporters.two_hop_closed_form(links_small, mu, nu)) < 1e-15


def test_one_hop_backward_is_dagger_of_link(links_small):
    for mu in range(4):
        n = [0, 0, 0, 0]
        n[mu] = -1
        w = transporters.transporter(links_small, tuple(n))
        assert np.allclose(w, dag(shift(links_small[mu], n)), atol=1e-15)


def test_transporter_hermiticity_and_norm(links_small):
    for n in all_offsets():
        w = transporters.transporter(links_small, n)
        back = transporters.transporter(links_small, tuple(-v for v in n))
        # W(x+n, x) = W(x, x+n)^dag
        assert np.allclose(shift(back, n), dag(w), atol=1e-14)
        assert transporters.max_spectral_norm(w) <= 1.0 + 1e-12


def test_transporter_gauge_covariance(links_small):
    g = synth.random_su3_field(DIMS_SMALL, seed=12)
    ug = synth.gauge_transform_links(links_small, g)
    for n in [(1, 0, 0, 0), (1, -1, 0, 0), (0, 1, -1, 1), (-1, 1, 1, -1), (1, 1, 1, 1)]:
        w = transporters.transporter(links_small, n)
        wg = transporters.transporter(ug, n)
        assert rel(wg, g @ w @ dag(shift(g, n))) < 1e-13


# ---------------------------------------------------------------- operator

MASS = 0.1


@pytest.mark.parametrize("mom", [(0, 0, 0, 0), (1, 0, 0, 0), (0, 2, 1, 3), (1, 1, 1, 1), (2, 0, 2, 0)])
def test_plane_waves_match_closed_form_symbol(mom):
    dims = (4, 4, 4, 4)
    u = synth.unit_links(dims)
    rng = np.random.default_rng(3)
    chi = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
    psi = synth.plane_wave(dims, mom, chi)
    k = 2 * np.pi * np.array(mom) / np.array(dims)
    sym = free.symbol(k, MASS)
    expect = synth.plane_wave(dims, mom, sym @ chi)
    out = dirac.apply(u, psi, MASS)
    # cancellations among O(1) stencil terms: measure against |psi|
    assert np.linalg.norm(out - expect) / np.linalg.norm(psi) < 1e-14
    assert np.allclose(free.fourier_sum(k, MASS), sym, atol=1e-14)


def test_doubler_corners_lifted_to_m_plus_2():
    for corner in itertools.product((0, 1), repeat=4):
        k = np.pi * np.array(corner, dtype=float)
        sym = free.symbol(k, MASS)
        expect = MASS if not any(corner) else MASS + 2.0
        assert np.allclose(sym, expect * np.eye(4), atol=1e-14)


def test_dense_spectrum_free_field_L2_L4():
    for dims in [(2, 2, 2, 2), (4, 2, 2, 4)]:
        u = synth.unit_links(dims)
        d = dirac.dense_matrix(u, MASS)
        ev = np.sort_complex(np.round(np.linalg.eigvals(d), 10))
        expect = []
        for mom in itertools.product(*[range(L) for L in dims]):
            k = 2 * np.pi * np.array(mom) / np.array(dims)
            lp, lm = free.eigenvalues(k, MASS)
            expect += [lp] * 6 + [lm] * 6
        expect = np.sort_complex(np.round(np.array(expect), 10))
        assert np.allclose(ev, expect, atol=1e-9)


def test_dense_matrix_matches_apply(links_small):
    psi = synth.gaussian_spinor(DIMS_SMALL, seed=13)
    d = dirac.dense_matrix(links_small, MASS)
    assert rel(d @ psi.reshape(-1), dirac.apply(links_small, psi, MASS).reshape(-1)) < 1e-14


def test_gamma5_hermiticity(links_small):
    psi = synth.gaussian_spinor(DIMS_SMALL, seed=14)
    chi = synth.gaussian_spinor(DIMS_SMALL, seed=15)
    dpsi = dirac.apply(links_small, psi, MASS)
    ddag_chi = dirac.apply_dag(links_small, chi, MASS)
    lhs = np.vdot(chi, dpsi)
    rhs = np.vdot(ddag_chi, psi)
    assert abs(lhs - rhs) / abs(lhs) < 1e-13
    assert rel(ddag_chi, dirac.apply_gamma5_sandwich(links_small, chi, MASS)) < 1e-13


def test_gauge_covariance(links_small):
    g = synth.random_su3_field(DIMS_SMALL, seed=16)
    ug = synth.gauge_transform_links(links_small, g)
    psi = synth.gaussian_spinor(DIMS_SMALL, seed=17)
    lhs = dirac.apply(ug, synth.gauge_transform_spinor(psi, g), MASS)
    rhs = synth.gauge_transform_spinor(dirac.apply(links_small, psi, MASS), g)
    assert rel(lhs, rhs) < 1e-13


def test_constants_annihilated_by_laplacian():
    dims = (3, 2, 4, 2)
    u = synth.unit_links(dims)
    v = np.arange(12).reshape(4, 3) * (1 + 0.5j)
    const = np.broadcast_to(v, synth.lattice_shape(dims) + (4, 3)).copy()
    # the stencil terms (O(1)) cancel down to m*const: measure against |const|
    assert np.linalg.norm(dirac.apply(u, const, MASS) - MASS * const) / np.linalg.norm(const) < 1e-14
    g = synth.random_su3_field(dims, seed=18)
    upure = synth.gauge_transform_links(u, g)
    gv = synth.gauge_transform_spinor(const, g)
    assert np.linalg.norm(dirac.apply(upure, gv, MASS) - MASS * gv) / np.linalg.norm(gv) < 1e-13


def test_agrees_with_factorized_formulation():
    dims = (4, 3, 2, 3)
    u = synth.gauge_links(dims, 0.4, seed=19)
    psi = synth.gaussian_spinor(dims, seed=20)
    assert rel(dirac.apply(u, psi, 0.05), factorized.apply(u, psi, 0.05)) < 1e-13


def test_pointwise_apply_matches_whole_lattice(links_small):
    psi = synth.gaussian_spinor(DIMS_SMALL, seed=21)
    full = dirac.apply(links_small, psi, MASS)
    sites = np.array([[0, 0, 0, 0], [2, 1, 0, 2], [1, 2, 2, 1], [2, 2, 2, 2]])
    pt = dirac.apply_at(links_small, psi, MASS, sites)
    for i, (x, y, z, t) in enumerate(sites):
        assert np.allclose(pt[i], full[t, z, y, x], atol=1e-13)


def test_pointwise_apply_dag_matches_whole_lattice(links_small):
    """The sampled-site D^dag (from D(y,x)^dag, links around x - n) equals the
    whole-lattice D^dag, which the gamma5-hermiticity pin ties to D."""
    psi = synth.gaussian_spinor(DIMS_SMALL, seed=22)
    full = dirac.apply_dag(links_small, psi, MASS)
    sites = np.array([[0, 0, 0, 0], [2, 1, 0, 2], [1, 2, 2, 1], [2, 2, 2, 2], [0, 2, 1, 2]])
    pt = dirac.apply_dag_at(links_small, psi, MASS, sites)
    for i, (x, y, z, t) in enumerate(sites):
        assert np.allclose(pt[i], full[t, z, y, x], atol=1e-13)
    # and it is not the sampled D: the two differ on random links
    assert not np.allclose(pt, dirac.apply_at(links_small, psi, MASS, sites), atol=1e-3)
