"""One step of APE link smearing (Sec. 5.1, Eq. def_ape).

TEST INFRASTRUCTURE ONLY (see the package docstring).

    V_mu(x) = P_SU(3){ (1 - alpha) 1
                       + (alpha/6) sum_{+-nu != mu} U_nu(x) U_mu(x+nu) U_nu(x+mu)^dag U_mu(x)^dag }
              U_mu(x)

The sum runs over the six directions +-nu orthogonal to mu.  A link "in
direction -nu" at y is the step y -> y - nu-hat, i.e. U_{-nu}(y) =
U_nu(y - nu-hat)^dag, so the -nu term reads

    U_nu(x-nu)^dag U_mu(x-nu) U_nu(x-nu+mu) U_mu(x)^dag.

Each term is a closed loop at x (a plaquette through x that contains the link
U_mu(x), traversed so that it ends with U_mu(x)^dag).  The paper uses
alpha = 0.72.

Parity: pinned (alpha = 0 and pure-gauge links leave U unchanged, gauge
covariance, and a closed form for links in a diagonal U(1) embedding,
computed from the link phases with scalar arithmetic).
"""
from __future__ import annotations

import numpy as np

from .lattice import dag
from .projection import project_sun
from .transporters import whole_lattice

ALPHA_PAPER = 0.72


def _unit(mu, s=1):
    e = [0, 0, 0, 0]
    e[mu] = s
    return e


def _add(a, b):
    return [a[i] + b[i] for i in range(4)]


def staple_loops(U, mu, get=whole_lattice):
    """sum over +-nu != mu of the closed loops of Eq. def_ape at every site."""
    o = [0, 0, 0, 0]
    umu_dag = dag(get(U[mu], o))
    acc = None
    for nu in range(4):
        if nu == mu:
            continue
        em, en, enm = _unit(mu), _unit(nu), _unit(nu, -1)
        # +nu: U_nu(x) U_mu(x+nu) U_nu(x+mu)^dag U_mu(x)^dag
        plus = get(U[nu], o) @ get(U[mu], en) @ dag(get(U[nu], em)) @ umu_dag
        # -nu: U_nu(x-nu)^dag U_mu(x-nu) U_nu(x-nu+mu) U_mu(x)^dag
        minus = dag(get(U[nu], enm)) @ get(U[mu], enm) @ get(U[nu], _add(enm, em)) @ umu_dag
        term = plus + minus
        acc = term if acc is None else acc + term
    return acc


def ape_link(U, mu, alpha, get=whole_lattice):
    """V_mu(x) of Eq. def_ape (at every site, or at the getter's sites)."""
    eye = np.eye(3, dtype=np.complex128)
    m = (1.0 - alpha) * eye + (alpha / 6.0) * staple_loops(U, mu, get)
    return project_sun(m) @ get(U[mu], [0, 0, 0, 0])


def ape(U, alpha=ALPHA_PAPER):
    """One APE step on the whole lattice; U[mu, t, z, y, x, 3, 3]."""
    return np.stack([ape_link(U, mu, alpha) for mu in range(4)])
