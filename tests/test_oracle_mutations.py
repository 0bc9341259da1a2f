"""Planted mistakes in the oracle (on the CPU) must each fail at least one of
the oracle's pins.

Each case below patches one oracle function with a plausible error (a
transposed transporter, a sign, a missing dagger, a wrong site, a dropped
path, a factor, a broken gamma basis, a missing mass term, a gradient chain
rule with a dagger dropped) and runs the pins of tests/test_oracle_*.py
against the patched oracle; the case passes only if some pin rejects it.
The unpatched oracle passes every pin (first test).  Nothing here touches
the GPU library."""
import inspect

import numpy as np
import pytest

import synth
from oracle import constants, dirac, factorized, free, gamma, grad, transporters, ultralocal, production, clover
from oracle.lattice import dag

from tests import test_oracle_constants as TC
from tests import test_oracle_operator as TO
from tests import test_oracle_solver_grad as TG


def _pins():
    links = synth.gauge_links(TO.DIMS_SMALL, 0.5, seed=11)
    gs = (synth.gauge_links(TG.DIMS_G, 0.4, seed=41), synth.gaussian_spinor(TG.DIMS_G, seed=42),
          synth.gaussian_spinor(TG.DIMS_G, seed=43))
    return [
        ("gamma algebra", TO.test_gamma_clifford_and_hermitian),
        ("path counts", TO.test_path_counts),
        ("unit links give W = 1", TO.test_unit_links_give_identity_transporters),
        ("two-hop closed form", lambda: TO.test_two_hop_closed_form(links)),
        ("one-hop backward = link^dag", lambda: TO.test_one_hop_backward_is_dagger_of_link(links)),
        ("W hermiticity and norm", lambda: TO.test_transporter_hermiticity_and_norm(links)),
        ("W gauge covariance", lambda: TO.test_transporter_gauge_covariance(links)),
        ("App. C Laplacian", TC.test_laplacian_matches_appC_table),
        ("App. C derivative", TC.test_x_derivative_matches_appC_table),
        ("Tab. rholambda", TC.test_class_coefficients_match_tab_rholambda),
        ("plane waves", lambda: [TO.test_plane_waves_match_closed_form_symbol(m)
                                 for m in ((1, 0, 0, 0), (0, 2, 1, 3))]),
        ("doublers at m + 2", TO.test_doubler_corners_lifted_to_m_plus_2),
        ("gamma5-hermiticity", lambda: TO.test_gamma5_hermiticity(links)),
        ("gauge covariance", lambda: TO.test_gauge_covariance(links)),
        ("constants annihilated", TO.test_constants_annihilated_by_laplacian),
        ("factorised formulation", TO.test_agrees_with_factorized_formulation),
        ("psi gradient by differences", lambda: TG.test_psi_gradient_central_difference(gs)),
        ("link gradient by differences", lambda: TG.test_link_gradient_central_difference(gs)),
    ]


def _first_failing_pin():
    for name, pin in _pins():
        try:
            pin()
        except Exception:  # an assertion, or the mistake breaking a shape
            return name
    return None


def _patch(monkeypatch, name, fn, modules):
    for m in modules:
        if hasattr(m, name):
            monkeypatch.setattr(m, name, fn)


# ---------------------------------------------------------------- mistakes
def _transposed_w(mp):
    orig = transporters.transporter

    def bad(U, n, get=transporters.whole_lattice):
        return np.swapaxes(orig(U, n, get), -1, -2)
    _patch(mp, "transporter", bad, [transporters, dirac, ultralocal, production])


def _weights_mutation(mp, change):
    orig = constants.operator_weights

    def bad(mass):
        lam, rho = orig(mass)
        return change(lam, rho, mass)
    _patch(mp, "operator_weights", bad, [constants, dirac, free, grad, production])


def _derivative_sign(mp):
    _weights_mutation(mp, lambda lam, rho, m: (lam, {n: -r for n, r in rho.items()}))


def _laplacian_factor(mp):
    def change(lam, rho, m):
        return {n: (2.0 * (v - m) + m if not any(n) else 2.0 * v) for n, v in lam.items()}, rho
    _weights_mutation(mp, change)


def _missing_mass(mp):
    _weights_mutation(mp, lambda lam, rho, m: ({n: (v - m if not any(n) else v) for n, v in lam.items()}, rho))


def _backward_no_dagger(mp):
    orig = transporters.link_step

    def bad(U, mu, s, get, d):
        return dag(orig(U, mu, s, get, d)) if s < 0 else orig(U, mu, s, get, d)
    _patch(mp, "link_step", bad, [transporters, grad])


def _backward_wrong_site(mp):
    def bad(U, mu, s, get, d):
        return get(U[mu], d) if s > 0 else dag(get(U[mu], d))
    _patch(mp, "link_step", bad, [transporters, grad])


def _dropped_path(mp):
    orig = transporters.path_orderings

    def bad(n):
        o = orig(n)
        return o[:-1] if len(o) > 1 else o
    _patch(mp, "path_orderings", bad, [transporters, grad])


def _gamma_basis(mp):
    orig = gamma.gammas

    def bad():
        g = orig()
        return [g[0], g[0], g[2], g[3]]
    _patch(mp, "gammas", bad, [gamma, dirac, free, factorized, clover])


def _gradient_dagger(mp):
    # the chain rule for a product with the left factor not daggered
    src = inspect.getsource(grad.grad_links)
    assert "g = dag(left) @ g" in src
    ns = dict(vars(grad))
    exec(compile(src.replace("g = dag(left) @ g", "g = left @ g"), "<planted>", "exec"), ns)
    mp.setattr(grad, "grad_links", ns["grad_links"])


MISTAKES = {
    "transposed transporter": _transposed_w,
    "derivative sign": _derivative_sign,
    "Laplacian factor 2": _laplacian_factor,
    "mass term dropped": _missing_mass,
    "backward step without dagger": _backward_no_dagger,
    "backward step at the wrong site": _backward_wrong_site,
    "one path dropped from the average": _dropped_path,
    "gamma_y = gamma_x": _gamma_basis,
    "gradient chain rule without a dagger": _gradient_dagger,
}


def test_unpatched_oracle_passes_every_pin():
    assert _first_failing_pin() is None


@pytest.mark.parametrize("mistake", list(MISTAKES))
def test_planted_mistake_fails_a_pin(monkeypatch, mistake):
    MISTAKES[mistake](monkeypatch)
    assert _first_failing_pin() is not None, f"no pin rejects: {mistake}"
