"""Pins for the oracle's stencil constants (no GPU).

The oracle derives its weights from the momentum-space symbols by inverse DFT;
here they are checked against what the paper prints in position space
(App. C stencil tables, Tab. rholambda) and against the conditions of Sec. 8.
"""
import itertools
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import constants
from oracle.lattice import all_offsets, hops

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_table(name):
    rows, divisor = [], None
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("divisor"):
                divisor = int(line.split()[1])
                continue
            rows.append([int(v) for v in line.split()])
    assert divisor is not None and len(rows) == 9 and all(len(r) == 9 for r in rows)
    w = np.zeros((3, 3, 3, 3), dtype=object)  # [nx+1, ny+1, nz+1, nt+1]
    for brow in range(3):          # n_t
        for line in range(3):      # n_y
            r = rows[3 * brow + line]
            for bcol in range(3):  # n_z
                for col in range(3):  # n_x
                    w[col, line, bcol, brow] = Fraction(r[3 * bcol + col], divisor)
    return w


def _read_rholambda():
    out = {}
    with open(os.path.join(GOLDEN, "tab_rholambda.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            name, wil, bri = line.split()
            out[name] = (Fraction(wil), Fraction(bri))
    return out


def test_laplacian_matches_appC_table():
    derived = constants.laplacian_weights()
    table = _read_table("appC_lap_bri.txt")
    for idx in itertools.product(range(3), repeat=4):
        assert constants.as_fraction(derived[idx]) == table[idx], idx
        assert abs(derived[idx] - float(table[idx])) < 1e-14


def test_x_derivative_matches_appC_table():
    derived = constants.derivative_weights()[0]
    table = _read_table("appC_der_iso_x.txt")
    for idx in itertools.product(range(3), repeat=4):
        assert constants.as_fraction(derived[idx]) == table[idx], idx


def test_other_derivatives_are_rotations_of_x():
    der = constants.derivative_weights()
    for mu in range(1, 4):
        perm = list(range(4))
        perm[0], perm[mu] = perm[mu], perm[0]
        assert np.allclose(np.transpose(der[0], perm), der[mu], atol=1e-15)


def test_class_coefficients_match_tab_rholambda():
    lam_k, rho_k = constants.class_coefficients()
    tab = _read_rholambda()
    for k in range(5):
        assert lam_k[k] == tab[f"lambda{k}"][1], (k, lam_k[k])
    for k in range(1, 5):
        assert rho_k[k] == tab[f"rho{k}"][1], (k, rho_k[k])


def test_81_points_and_class_sizes():
    offs = all_offsets()
    assert len(offs) == 80 and len(set(offs)) == 80
    sizes = [sum(1 for n in offs if hops(n) == k) for k in range(1, 5)]
    assert [1] + sizes == [1, 8, 24, 32, 16]
    assert 1 + sum(sizes) == 81
    lap = constants.laplacian_weights()
    assert np.count_nonzero(np.abs(lap) > 0) == 81


@pytest.mark.parametrize("col", [0, 1])
def test_sec8_normalisation_conditions(col):
    """2 rho1 + 12 rho2 + 24 rho3 + 16 rho4 = 1 and the lambda sum rule, for the
    Wilson and the Brillouin columns of the table (Sec. 8)."""
    t = {k: v[col] for k, v in _read_rholambda().items()}
    assert 2 * t["rho1"] + 12 * t["rho2"] + 24 * t["rho3"] + 16 * t["rho4"] == 1
    assert t["lambda0"] + 8 * t["lambda1"] + 24 * t["lambda2"] + 32 * t["lambda3"] + 16 * t["lambda4"] == 0


def test_sec8_doubler_and_dispersion_conditions_from_derived():
    lam_k, rho_k = constants.class_coefficients()
    l0, l1, l2, l3, l4 = (lam_k[k] for k in range(5))
    assert l0 + 4 * l1 - 16 * l3 - 16 * l4 == 2
    assert l0 - 8 * l2 + 16 * l4 == 2
    assert l0 - 4 * l1 + 16 * l3 - 16 * l4 == 2
    assert l0 - 8 * l1 + 24 * l2 - 32 * l3 + 16 * l4 == 2
    assert 12 * rho_k[2] + 48 * rho_k[3] + 48 * rho_k[4] - 1 == 0
    assert l0 + 8 * l1 + 24 * l2 + 32 * l3 + 16 * l4 == 0


def test_laplacian_annihilates_constants():
    assert abs(constants.laplacian_weights().sum()) < 1e-14
    assert np.allclose(constants.derivative_weights().sum(axis=(1, 2, 3, 4)), 0.0, atol=1e-15)


def test_symbol_values_at_special_momenta():
    """Lap^bri = -4 on the whole Brillouin-zone boundary (Sec. 4.1) and 0 at k = 0;
    the derivative symbol vanishes wherever any component is pi."""
    rng = np.random.default_rng(7)
    for _ in range(20):
        k = rng.uniform(-np.pi, np.pi, size=4)
        k[rng.integers(4)] = np.pi
        assert abs(constants.lap_bri_symbol(k) + 4.0) < 1e-14
        for mu in range(4):
            assert abs(constants.der_iso_symbol(k, mu)) < 1e-14 or abs(k[mu]) != np.pi
    assert abs(constants.lap_bri_symbol(np.zeros(4))) < 1e-15
