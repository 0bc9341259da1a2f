"""The generic ultralocal class of Wilson-type operators (Sec. 8, Tab. rholambda).

The Brillouin operator is one member of the class

    D(x,y) = sum_mu gamma_mu rho_mu(x-y) + lambda(x-y),

supported on y = x + n, n in {-1,0,1}^4, and made covariant with the same
path-averaged transporters W(x, x+n) (Sec. 5.1).  An offset with k non-zero
components carries

    lambda(n) = lambda_k,      rho_mu(n) = rho_k n_mu,

so a member is fixed by nine numbers (lambda_0..lambda_4, rho_1..rho_4), and

    (D psi)(x) = (lambda_0 + m) psi(x)
               + sum_{n != 0} [lambda_k + rho_k sum_mu n_mu gamma_mu] W(x,x+n) psi(x+n).

A table here is that tuple, in this order.

Readings (the printed formulas of Sec. 8 are garbled in two places):
* every offset is counted once in each sum.  The normalisation conditions of
  Sec. 8, 2 rho_1 + 12 rho_2 + 24 rho_3 + 16 rho_4 = 1 and
  lambda_0 + 8 lambda_1 + 24 lambda_2 + 32 lambda_3 + 16 lambda_4 = 0, count
  8, 24, 32, 16 offsets of 1..4 hops, and the Brillouin column of the table
  then reproduces the position-space Laplacian of App. C;
* the lambda sums add the two directions (the printed differences would make
  the Laplacian odd, and then no column of the table would satisfy the
  lambda condition).

The adjoint is written from D^dag(x,y) = D(y,x)^dag; gamma5-hermiticity is
checked by the tests, not used.

Parity: pinned (the Wilson column against the hopping form of the Wilson
operator in Sec. 1 with 1/(2 kappa) = 4 + m; the Brillouin column against
``oracle.dirac``, whose weights come from the momentum-space product forms;
the free-field Fourier sum against closed forms built from elementary
symmetric polynomials, and for the two exact columns against the textbook
Wilson symbol and the paper's Brillouin symbol; the free spectrum at L = 2:
Wilson branches at 0, 2, 4, 6, 8 with multiplicities 1, 4, 6, 4, 1 (Sec. 4.2)
and the Brillouin doublers all at 2 (Sec. 8); gamma5-hermiticity and gauge
covariance for the decimal hypercube column).
"""
from __future__ import annotations

import numpy as np

from .dirac import _colour, _spin, coefficient_matrix
from .lattice import all_offsets, dag, hops, shift
from .transporters import make_site_getter, transporter, whole_lattice

# lambda_0..lambda_4, rho_1..rho_4 of Tab. rholambda.
WILSON = (4.0, -0.5, 0.0, 0.0, 0.0, 0.5, 0.0, 0.0, 0.0)
BRILLOUIN = (240 / 128, -8 / 128, -4 / 128, -2 / 128, -1 / 128, 64 / 432, 16 / 432, 4 / 432, 1 / 432)
HYPERCUBE = (1.852720547, -0.060757866, -0.030036032, -0.015967620, -0.008426812,
             0.136846794, 0.032077284, 0.011058131, 0.004748991)


def weights(table, mass):
    """lambda(n) and rho_mu(n) for n = 0 and the 80 offsets (lambda(0) includes m)."""
    lam_k = [float(v) for v in table[:5]]
    rho_k = [0.0] + [float(v) for v in table[5:9]]
    lam = {(0, 0, 0, 0): lam_k[0] + mass}
    rho = {(0, 0, 0, 0): np.zeros(4)}
    for n in all_offsets():
        k = hops(n)
        lam[n] = lam_k[k]
        rho[n] = rho_k[k] * np.array(n, dtype=float)
    return lam, rho


def _apply(U, psi, lam, rho, get, psi_here):
    out = lam[(0, 0, 0, 0)] * psi_here
    for n in all_offsets():
        w = transporter(U, n, get)
        out = out + _spin(coefficient_matrix(lam, rho, n), _colour(w, get(psi, n)))
    return out


def apply(U, psi, mass, table):
    """D psi on the whole lattice; psi has shape (Lt, Lz, Ly, Lx, 4, 3)."""
    lam, rho = weights(table, mass)
    return _apply(U, psi, lam, rho, whole_lattice, psi)


def apply_at(U, psi, mass, table, sites):
    """(D psi)(x) at the sampled sites (N, 4) = (x, y, z, t); shape (N, 4, 3)."""
    dims = (psi.shape[3], psi.shape[2], psi.shape[1], psi.shape[0])
    get = make_site_getter(sites, dims)
    lam, rho = weights(table, mass)
    return _apply(U, psi, lam, rho, get, get(psi, (0, 0, 0, 0)))


def apply_dag(U, psi, mass, table):
    """D^dag psi from D^dag(x,y) = D(y,x)^dag."""
    lam, rho = weights(table, mass)
    out = np.conj(lam[(0, 0, 0, 0)]) * psi
    for n in all_offsets():
        back = tuple(-v for v in n)
        w_from = shift(transporter(U, n), back)  # W(x-n, x) at every x
        cd = dag(coefficient_matrix(lam, rho, n))
        out = out + _spin(cd, _colour(dag(w_from), shift(psi, back)))
    return out


def fourier_sum(k, mass, table):
    """Free-field symbol sum_n C(n) e^{i k.n} (4x4) at one momentum k."""
    lam, rho = weights(table, mass)
    out = lam[(0, 0, 0, 0)] * np.eye(4, dtype=np.complex128)
    for n in all_offsets():
        out = out + coefficient_matrix(lam, rho, n) * np.exp(1j * np.dot(k, n))
    return out


def dense_matrix(U, mass, table):
    """The operator as a dense (12V x 12V) matrix, column by column (tiny lattices)."""
    lt, lz, ly, lx = U.shape[1:5]
    nv = lx * ly * lz * lt * 12
    out = np.zeros((nv, nv), dtype=np.complex128)
    e = np.zeros(nv, dtype=np.complex128)
    for j in range(nv):
        e[:] = 0
        e[j] = 1
        out[:, j] = apply(U, e.reshape(lt, lz, ly, lx, 4, 3), mass, table).reshape(-1)
    return out
