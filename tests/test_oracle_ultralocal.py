"""Pins of the generic ultralocal class oracle (Sec. 8, Tab. rholambda): the
Wilson column against the hopping form of the Wilson operator (Sec. 1), the
Brillouin column against the independently derived Brillouin oracle, the
free symbol against closed forms, and the free spectra at L = 2."""
import itertools
import os
from fractions import Fraction

import numpy as np
import pytest

import synth
from oracle import clover, dirac, free, production, smearing, ultralocal
from oracle.gamma import gamma5, gammas

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
MASS = 0.1


def rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def _read(name, col):
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            parts = line.split()
            out[parts[0]] = parts[1 + col]
    return out


def _as_table(d, conv):
    return tuple(conv(d[f"lambda{k}"]) for k in range(5)) + tuple(conv(d[f"rho{k}"]) for k in range(1, 5))


def test_tables_match_fixtures():
    assert ultralocal.WILSON == _as_table(_read("tab_rholambda.txt", 0), lambda s: float(Fraction(s)))
    assert ultralocal.BRILLOUIN == _as_table(_read("tab_rholambda.txt", 1), lambda s: float(Fraction(s)))
    assert ultralocal.HYPERCUBE == _as_table(_read("tab_rholambda_hypercube.txt", 0), float)


def test_hypercube_column_satisfies_sec8_conditions():
    """The normalisation conditions hold to the nine printed digits."""
    l0, l1, l2, l3, l4, r1, r2, r3, r4 = ultralocal.HYPERCUBE
    assert abs(2 * r1 + 12 * r2 + 24 * r3 + 16 * r4 - 1) < 5e-8
    assert abs(l0 + 8 * l1 + 24 * l2 + 32 * l3 + 16 * l4) < 5e-8


@pytest.fixture(scope="module")
def links():
    dims = (3, 3, 2, 4)
    return dims, synth.gauge_links(dims, 0.5, 8301)


def _wilson_hopping(u, psi, mass):
    """Sec. 1: D = 1/2 sum_mu {(gamma_mu - 1) U_mu(x) psi(x+mu) - (gamma_mu + 1) U_mu(x-mu)^dag psi(x-mu)}
    + 1/(2 kappa) psi(x), with 1/(2 kappa) = 4 + m."""
    g = gammas()
    one = np.eye(4)
    out = (4.0 + mass) * psi
    for mu in range(4):
        ax = 3 - mu
        fwd = np.einsum("...ab,...sb->...sa", u[mu], np.roll(psi, -1, axis=ax))
        ub = np.roll(u[mu], 1, axis=ax)  # U_mu(x - mu)
        bwd = np.einsum("...ba,...sb->...sa", ub.conj(), np.roll(psi, 1, axis=ax))
        out = out + 0.5 * np.einsum("st,...tc->...sc", g[mu] - one, fwd)
        out = out - 0.5 * np.einsum("st,...tc->...sc", g[mu] + one, bwd)
    return out


def test_wilson_column_is_the_hopping_form(links):
    dims, u = links
    psi = synth.gaussian_spinor(dims, 8302)
    got = ultralocal.apply(u, psi, MASS, ultralocal.WILSON)
    assert rel(got, _wilson_hopping(u, psi, MASS)) < 1e-14


def test_brillouin_column_is_the_brillouin_operator(links):
    dims, u = links
    psi = synth.gaussian_spinor(dims, 8303)
    assert rel(ultralocal.apply(u, psi, MASS, ultralocal.BRILLOUIN), dirac.apply(u, psi, MASS)) < 1e-13
    assert rel(ultralocal.apply_dag(u, psi, MASS, ultralocal.BRILLOUIN), dirac.apply_dag(u, psi, MASS)) < 1e-13


def _esym(vals, k):
    """Elementary symmetric polynomial e_k."""
    return sum(np.prod(c) for c in itertools.combinations(vals, k)) if k else 1.0


def test_fourier_sum_closed_forms():
    """Each coefficient alone: lambda_k -> e_k(2 cos k_1, ..., 2 cos k_4);
    rho_k -> sum_mu gamma_mu 2i sin k_mu e_{k-1}(2 cos k_nu, nu != mu)."""
    g = gammas()
    rng = np.random.default_rng(8304)
    for _ in range(6):
        k = rng.uniform(-np.pi, np.pi, 4)
        c2 = 2 * np.cos(k)
        for i in range(9):
            t = [0.0] * 9
            t[i] = 1.0
            got = ultralocal.fourier_sum(k, 0.0, t)
            if i < 5:
                want = _esym(c2, i) * np.eye(4)
            else:
                kk = i - 4
                want = sum(g[mu] * 2j * np.sin(k[mu]) * _esym([c2[nu] for nu in range(4) if nu != mu], kk - 1)
                           for mu in range(4))
            assert np.abs(got - want).max() < 1e-13, (i, k)
        wil = (4 + MASS - np.cos(k).sum()) * np.eye(4) + sum(1j * np.sin(k[mu]) * g[mu] for mu in range(4))
        assert np.abs(ultralocal.fourier_sum(k, MASS, ultralocal.WILSON) - wil).max() < 1e-13
        assert np.abs(ultralocal.fourier_sum(k, MASS, ultralocal.BRILLOUIN) - free.symbol(k, MASS)).max() < 1e-13


def test_plane_waves_hypercube():
    dims = (4, 3, 2, 5)
    u = synth.unit_links(dims)
    rng = np.random.default_rng(8305)
    for mom in [(1, 0, 1, 2), (3, 2, 1, 4), (0, 1, 0, 0)]:
        k = np.array([2 * np.pi * mom[mu] / dims[mu] for mu in range(4)])
        chi = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        out = ultralocal.apply(u, synth.plane_wave(dims, mom, chi), MASS, ultralocal.HYPERCUBE)
        want = synth.plane_wave(dims, mom, ultralocal.fourier_sum(k, MASS, ultralocal.HYPERCUBE) @ chi)
        assert rel(out, want) < 1e-13


@pytest.mark.parametrize("table,branches", [
    (ultralocal.WILSON, {0: 1, 2: 4, 4: 6, 6: 4, 8: 1}),
    (ultralocal.BRILLOUIN, {0: 1, 2: 15}),
])
def test_free_spectrum_at_L2(table, branches):
    """Unit links on 2^4: momenta {0, pi}^4 only.  Wilson: the 16 species at
    0, 2, 4, 6, 8 with multiplicities 1, 4, 6, 4, 1 (Sec. 4.2); Brillouin: every
    doubler lifted to 2 (the equal-lift conditions of Sec. 8).  Each species
    carries 4 spins x 3 colours."""
    d = ultralocal.dense_matrix(synth.unit_links((2, 2, 2, 2)), 0.0, table)
    ev = np.linalg.eigvals(d)
    assert np.abs(ev.imag).max() < 1e-12
    vals, counts = np.unique(np.round(ev.real, 9), return_counts=True)
    assert dict(zip(vals.tolist(), counts.tolist())) == {float(k): 12 * v for k, v in branches.items()}


def test_hypercube_gamma5_hermiticity_and_covariance(links):
    dims, u = links
    g5 = gamma5()
    psi = synth.gaussian_spinor(dims, 8306)
    t = ultralocal.HYPERCUBE
    sand = np.einsum("st,...tc->...sc", g5, ultralocal.apply(u, np.einsum("st,...tc->...sc", g5, psi), MASS, t))
    assert rel(ultralocal.apply_dag(u, psi, MASS, t), sand) < 1e-13
    g = synth.random_su3_field(dims, seed=8307)
    lhs = ultralocal.apply(synth.gauge_transform_links(u, g), synth.gauge_transform_spinor(psi, g), MASS, t)
    rhs = synth.gauge_transform_spinor(ultralocal.apply(u, psi, MASS, t), g)
    assert rel(lhs, rhs) < 1e-13


def test_apply_at_matches_whole_lattice(links):
    dims, u = links
    psi = synth.gaussian_spinor(dims, 8308)
    t = ultralocal.HYPERCUBE
    full = ultralocal.apply(u, psi, MASS, t)
    sites = np.array([[0, 0, 0, 0], [2, 1, 1, 3], [1, 2, 0, 2]])
    got = ultralocal.apply_at(u, psi, MASS, t, sites)
    want = np.stack([full[s[3], s[2], s[1], s[0]] for s in sites])
    assert rel(got, want) < 1e-14


def test_production_form_with_wilson_table_is_wilson_clover(links):
    """With back-projected transporters and the clover term, the Wilson column
    gives the clover-improved Wilson operator of Sec. 1 (one-hop transporters
    are the links themselves, already in SU(3))."""
    dims, u = links
    psi = synth.gaussian_spinor(dims, 8309)
    got = production.apply(u, psi, MASS, csw=1.0, table=ultralocal.WILSON)
    want = _wilson_hopping(u, psi, MASS) + clover.apply_clover(u, psi, 1.0)
    assert rel(got, want) < 1e-14


def test_production_form_with_table_free_limit_and_hermiticity():
    dims = (3, 2, 3, 3)
    psi = synth.gaussian_spinor(dims, 8310)
    t = ultralocal.HYPERCUBE
    unit = synth.unit_links(dims)
    assert rel(production.apply(unit, psi, MASS, table=t), ultralocal.apply(unit, psi, MASS, t)) < 1e-14
    u = smearing.ape(synth.gauge_links(dims, 0.4, 8311), 0.72)
    g5 = gamma5()
    sand = np.einsum("st,...tc->...sc", g5,
                     production.apply(u, np.einsum("st,...tc->...sc", g5, psi), MASS, table=t))
    assert rel(production.apply_dag(u, psi, MASS, table=t), sand) < 1e-13
    sites = np.array([[0, 0, 0, 0], [2, 1, 2, 1]])
    full = production.apply(u, psi, MASS, table=t)
    part = production.apply_at(u, psi, MASS, sites, table=t)
    for j, (x, y, z, tt) in enumerate(sites):
        assert np.abs(part[j] - full[tt, z, y, x]).max() < 1e-14
