"""The Brillouin Dirac operator, written out from its definition (FP64, numpy).

Eq. def_pref with c_SW = 0 and a = 1:

    D(x,y) = sum_mu gamma_mu d^iso_mu(x,y) - (1/2) Lap^bri(x,y) + m delta_{x,y}

with both stencils supported on y = x + n, n in {-1,0,1}^4, and made covariant
by the path-averaged transporter W(x, x+n) (Sec. 5.1).  Hence

    (D psi)(x) = sum_{n} C(n) W(x, x+n) psi(x+n),
    C(n) = lambda(n) + sum_mu rho_mu(n) gamma_mu,   W(x, x) = 1,

with lambda(n), rho_mu(n) the position-space weights of ``oracle.constants``
(lambda(0) includes m).  C acts on spin, W on colour.

The adjoint is written from its definition, D^dag(x,y) = D(y,x)^dag, i.e.

    (D^dag psi)(x) = sum_n C(n)^dag W(x-n, x)^dag psi(x-n),

with no use of gamma5-hermiticity (which the tests check separately).

Parity: pinned (free plane waves against the momentum-space symbol of
Eq. def_4Dbri and App. C, dense spectrum at L = 2 and 4, gamma5-hermiticity,
gauge covariance, constants annihilated, agreement with ``oracle.factorized``).
"""
from __future__ import annotations

import numpy as np

from .constants import operator_weights
from .gamma import gammas, gamma5
from .lattice import all_offsets, shift, dag
from .transporters import transporter, whole_lattice, make_site_getter

_I4 = np.eye(4, dtype=np.complex128)


def coefficient_matrix(lam, rho, n):
    """C(n) = lambda(n) 1 + sum_mu rho_mu(n) gamma_mu (4x4 spin matrix)."""
    g = gammas()
    c = lam[n] * _I4
    for mu in range(4):
        c = c + rho[n][mu] * g[mu]
    return c


def _colour(w, psi):
    return np.einsum("...ab,...sb->...sa", w, psi)


def _spin(c, psi):
    return np.einsum("st,...tc->...sc", c, psi)


def _apply(U, psi, mass, get, psi_here):
    lam, rho = operator_weights(mass)
    out = lam[(0, 0, 0, 0)] * psi_here
    for n in all_offsets():
        w = transporter(U, n, get)
        out = out + _spin(coefficient_matrix(lam, rho, n), _colour(w, get(psi, n)))
    return out


def apply(U, psi, mass):
    """D psi on the whole lattice; psi has shape (Lt, Lz, Ly, Lx, 4, 3)."""
    return _apply(U, psi, mass, whole_lattice, psi)


def apply_at(U, psi, mass, sites):
    """(D psi)(x) only at the sampled sites (N, 4) = (x, y, z, t): uses nothing
    but psi and the links inside x + {-1,0,1}^4 (plus one link layer for the
    backward steps).  Returns shape (N, 4, 3)."""
    dims = (psi.shape[3], psi.shape[2], psi.shape[1], psi.shape[0])
    get = make_site_getter(sites, dims)
    return _apply(U, psi, mass, get, get(psi, (0, 0, 0, 0)))


def apply_dag(U, psi, mass):
    """D^dag psi from D^dag(x,y) = D(y,x)^dag."""
    lam, rho = operator_weights(mass)
    out = np.conj(lam[(0, 0, 0, 0)]) * psi
    for n in all_offsets():
        back = tuple(-v for v in n)
        w_from = shift(transporter(U, n), back)  # W(x-n, x) at every x
        cd = dag(coefficient_matrix(lam, rho, n))
        out = out + _spin(cd, _colour(dag(w_from), shift(psi, back)))
    return out


def apply_dag_at(U, psi, mass, sites):
    """(D^dag psi)(x) only at the sampled sites (N, 4) = (x, y, z, t), from
    D^dag(x,y) = D(y,x)^dag: the term of offset n is C(n)^dag W(x-n, x)^dag
    psi(x-n), with W(x-n, x) enumerated from the links around x-n.  Returns
    shape (N, 4, 3)."""
    dims = (psi.shape[3], psi.shape[2], psi.shape[1], psi.shape[0])
    get = make_site_getter(sites, dims)
    lam, rho = operator_weights(mass)
    out = np.conj(lam[(0, 0, 0, 0)]) * get(psi, (0, 0, 0, 0))
    for n in all_offsets():
        back = tuple(-v for v in n)

        def get_back(field, d, back=back):
            return get(field, tuple(d[mu] + back[mu] for mu in range(4)))

        w_from = transporter(U, n, get_back)  # W(x-n, x) at every sampled x
        cd = dag(coefficient_matrix(lam, rho, n))
        out = out + _spin(cd, _colour(dag(w_from), get(psi, back)))
    return out


def apply_gamma5_sandwich(U, psi, mass):
    """gamma5 D gamma5 psi (used to check gamma5-hermiticity, Sec. 1)."""
    g5 = gamma5()
    return _spin(g5, apply(U, _spin(g5, psi), mass))


def site_index(dims, x, y, z, t):
    lx, ly, lz, _ = dims
    return x + lx * (y + ly * (z + lz * t))


def dense_matrix(U, mass):
    """The 12V x 12V matrix of D, row/column index 12*site + 3*spin + colour."""
    lt, lz, ly, lx = U.shape[1:5]
    dims = (lx, ly, lz, lt)
    v = lx * ly * lz * lt
    lam, rho = operator_weights(mass)
    d = np.zeros((12 * v, 12 * v), dtype=np.complex128)
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx),
                             indexing="ij")
    src = site_index(dims, x, y, z, t).reshape(-1)
    rows = (12 * src[:, None] + np.arange(12)[None, :])
    d[rows[:, :, None], rows[:, None, :]] += lam[(0, 0, 0, 0)] * np.eye(12)[None]
    for n in all_offsets():
        w = transporter(U, n).reshape(v, 3, 3)
        c = coefficient_matrix(lam, rho, n)
        blk = np.einsum("st,vab->vsatb", c, w).reshape(v, 12, 12)
        dst = site_index(dims, (x + n[0]) % lx, (y + n[1]) % ly, (z + n[2]) % lz,
                         (t + n[3]) % lt).reshape(-1)
        cols = 12 * dst[:, None] + np.arange(12)[None, :]
        d[rows[:, :, None], cols[:, None, :]] += blk
    return d


def flatten_spinor(psi):
    """Canonical (Lt,Lz,Ly,Lx,4,3) field -> vector with index 12*site + 3*s + c."""
    return psi.reshape(-1)
