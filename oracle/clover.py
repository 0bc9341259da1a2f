"""The clover term of Eq. def_pref: -(c_SW/2) sum_{mu<nu} sigma_{mu nu} F_{mu nu}.

TEST INFRASTRUCTURE ONLY (see the package docstring).

* sigma_{mu nu} = (i/2) [gamma_mu, gamma_nu] (Sec. 1), from ``oracle.gamma``;
* F_{mu nu} is the Hermitian clover-leaf field strength: with Q_{mu nu}(x)
  the sum of the four plaquettes in the (mu, nu) plane that start and end at
  x, all traversed in the same sense (mu before nu),

      F_{mu nu} = (Q_{mu nu} - Q_{mu nu}^dag) / (8 i),

  made traceless by subtracting tr(F)/3 (the reading adopted here: the field
  strength lives in the Lie algebra of SU(3); the paper only calls it the
  Hermitian clover-leaf tensor);
* the tree-level coefficient is c_SW = 1 (Sec. 5.3).

The term is a 12x12 matrix per site (index 3*spin + colour), Hermitian, and
acts on psi(x) only.

Parity: pinned (F = 0 for unit and pure-gauge links, Hermiticity and
tracelessness, gauge covariance F -> g F g^dag, a closed form for links in a
diagonal U(1) embedding from scalar phase arithmetic, sigma algebra checks).
"""
from __future__ import annotations

import numpy as np

from .gamma import gammas
from .lattice import dag
from .transporters import whole_lattice

CSW_TREE = 1.0


def sigma(mu, nu):
    g = gammas()
    return 0.5j * (g[mu] @ g[nu] - g[nu] @ g[mu])


def _e(mu, s=1):
    e = [0, 0, 0, 0]
    e[mu] = s
    return e


def _add(*vs):
    return [sum(v[i] for v in vs) for i in range(4)]


def leaves(U, mu, nu, get=whole_lattice):
    """Q_{mu nu}(x): the four plaquettes at x in the (mu, nu) plane."""
    o = [0, 0, 0, 0]
    pm, pn, mm, mn = _e(mu), _e(nu), _e(mu, -1), _e(nu, -1)
    Umu, Unu = U[mu], U[nu]
    # x -> x+mu -> x+mu+nu -> x+nu -> x
    q1 = get(Umu, o) @ get(Unu, pm) @ dag(get(Umu, pn)) @ dag(get(Unu, o))
    # x -> x+nu -> x+nu-mu -> x-mu -> x
    q2 = get(Unu, o) @ dag(get(Umu, _add(mm, pn))) @ dag(get(Unu, mm)) @ get(Umu, mm)
    # x -> x-mu -> x-mu-nu -> x-nu -> x
    q3 = dag(get(Umu, mm)) @ dag(get(Unu, _add(mm, mn))) @ get(Umu, _add(mm, mn)) @ get(Unu, mn)
    # x -> x-nu -> x-nu+mu -> x+mu -> x
    q4 = dag(get(Unu, mn)) @ get(Umu, mn) @ get(Unu, _add(mn, pm)) @ dag(get(Umu, o))
    return q1 + q2 + q3 + q4


def field_strength(U, mu, nu, get=whole_lattice):
    """Traceless Hermitian F_{mu nu}(x) = (Q - Q^dag)/(8i) - tr/3."""
    q = leaves(U, mu, nu, get)
    f = (q - dag(q)) / 8j
    tr = np.trace(f, axis1=-2, axis2=-1)
    return f - (tr / 3.0)[..., None, None] * np.eye(3)


def clover_matrix(U, csw=CSW_TREE, get=whole_lattice):
    """-(c_SW/2) sum_{mu<nu} sigma_{mu nu} (x) F_{mu nu}: (..., 12, 12)."""
    out = None
    for mu in range(4):
        for nu in range(mu + 1, 4):
            f = field_strength(U, mu, nu, get)
            term = np.einsum("st,...ab->...satb", sigma(mu, nu), f)
            term = term.reshape(f.shape[:-2] + (12, 12))
            out = term if out is None else out + term
    return -0.5 * csw * out


def apply_clover(U, psi, csw=CSW_TREE, get=whole_lattice):
    """The clover term times psi(x); psi has trailing shape (4, 3)."""
    c = clover_matrix(U, csw, get)
    flat = psi.reshape(psi.shape[:-2] + (12,))
    return np.einsum("...ij,...j->...i", c, flat).reshape(psi.shape)
