"""The paper's production form of the Brillouin operator (Sec. 5).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Eq. def_pref with all three ingredients of Sec. 5:

    (D psi)(x) = (lambda_0 + m) psi(x)
               + sum_{n != 0} C(n) W_SU3(x, x+n) psi(x+n)
               - (c_SW/2) sum_{mu<nu} sigma_{mu nu} F_{mu nu}(x) psi(x),

where
* the links are used as given (one APE step, ``oracle.smearing.ape``, is
  applied by the caller when the smeared operator is wanted);
* W_SU3(x, x+n) = P_SU(3){ average of the k! shortest-path products }
  (Sec. 5.1, "with subsequent backprojection to SU(3)", the projection of
  Sec. 5.2, ``oracle.projection.project_sun``);
* F_{mu nu} and sigma_{mu nu} are those of ``oracle.clover``, c_SW = 1 at tree
  level (Sec. 5.3).

The adjoint is written from D^dag(x,y) = D(y,x)^dag.

``table`` (optional) replaces the Brillouin coefficients by another member of
the generic class of Sec. 8 (``oracle.ultralocal``: lambda_0..4, rho_1..4);
the transporters and the clover term stay as above.

Parity: pinned through its parts (projection, smearing and clover modules)
and, for the whole operator, gamma5-hermiticity, gauge covariance, the free
limit (unit links: W_SU3 = 1, F = 0, so it equals the plain operator) and
the U(1)-embedding closed form of the projected transporters.
"""
from __future__ import annotations

import numpy as np

from .clover import CSW_TREE, apply_clover, clover_matrix
from .constants import operator_weights
from .dirac import coefficient_matrix, _colour, _spin
from .lattice import all_offsets, dag, shift
from .projection import project_sun
from .transporters import make_site_getter, transporter, whole_lattice
from . import ultralocal


def transporter_su3(U, n, get=whole_lattice):
    """P_SU(3) of the path average W(x, x+n)."""
    return project_sun(transporter(U, n, get))


def _weights(mass, table):
    return operator_weights(mass) if table is None else ultralocal.weights(table, mass)


def _apply(U, psi, mass, csw, get, psi_here, table=None):
    lam, rho = _weights(mass, table)
    out = lam[(0, 0, 0, 0)] * psi_here
    for n in all_offsets():
        w = transporter_su3(U, n, get)
        out = out + _spin(coefficient_matrix(lam, rho, n), _colour(w, get(psi, n)))
    if csw != 0.0:
        out = out + apply_clover(U, psi_here, csw, get)
    return out


def apply(U, psi, mass, csw=CSW_TREE, table=None):
    """D psi on the whole lattice; psi has shape (Lt, Lz, Ly, Lx, 4, 3)."""
    return _apply(U, psi, mass, csw, whole_lattice, psi, table)


def apply_at(U, psi, mass, sites, csw=CSW_TREE, table=None):
    """(D psi)(x) at the sampled sites (N, 4) = (x, y, z, t); shape (N, 4, 3)."""
    dims = (psi.shape[3], psi.shape[2], psi.shape[1], psi.shape[0])
    get = make_site_getter(sites, dims)
    return _apply(U, psi, mass, csw, get, get(psi, (0, 0, 0, 0)), table)


def apply_dag(U, psi, mass, csw=CSW_TREE, table=None):
    """D^dag psi from D^dag(x,y) = D(y,x)^dag."""
    lam, rho = _weights(mass, table)
    out = np.conj(lam[(0, 0, 0, 0)]) * psi
    for n in all_offsets():
        back = tuple(-v for v in n)
        w_from = shift(transporter_su3(U, n), back)  # W(x-n, x) at every x
        cd = dag(coefficient_matrix(lam, rho, n))
        out = out + _spin(cd, _colour(dag(w_from), shift(psi, back)))
    if csw != 0.0:
        c = dag(clover_matrix(U, csw))
        flat = psi.reshape(psi.shape[:-2] + (12,))
        out = out + np.einsum("...ij,...j->...i", c, flat).reshape(psi.shape)
    return out
