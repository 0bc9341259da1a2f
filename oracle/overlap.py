"""The overlap operator with the Brillouin kernel (Sec. 7, Eqs. def_over and
def_mass), dense and exact, for small lattices.

TEST INFRASTRUCTURE ONLY (see the package docstring).

    D_ov = rho [1 + gamma5 sign(H)],   H = gamma5 D_kn(-rho)       (Eq. def_over, a = 1)
    D_ov,m = (1 - m/(2 rho)) D_ov + m                               (Eq. def_mass)

with D_kn(-rho) the kernel operator at mass -rho (here the Brillouin operator
of ``oracle.dirac`` or the production form of ``oracle.production``) and
0 < rho < 2 (canonical rho = 1).  H is Hermitian (gamma5-hermiticity), so
sign(H) = V sign(Lambda) V^dag from its eigen-decomposition, and H^2 =
D^dag D.  The extremal eigenvalues of A = D^dag D are what the Lanczos
process estimates (the Ritz values of Sec. 7.3).

Everything is dense (12V x 12V), so only tiny lattices (V <= 4^4).

Parity: pinned (sign(H)^2 = 1, the Ginsparg-Wilson relation
gamma5 D + D gamma5 = D gamma5 D / rho, the spectrum on the circle of radius
rho around rho, gamma5-hermiticity of D_ov, and the free-field closed form
from the momentum-space symbol of ``oracle.free``).
"""
from __future__ import annotations

import numpy as np

from . import dirac
from .gamma import gamma5

RHO = 1.0


def gamma5_full(nsites):
    """gamma5 on the 12V-dimensional space (index 12*site + 3*spin + colour)."""
    return np.kron(np.eye(nsites), np.kron(gamma5(), np.eye(3)))


def kernel_matrix(U, rho=RHO, dense=None):
    """D_kn(-rho) as a dense matrix (the Brillouin operator at mass -rho), or
    the given dense kernel at mass 0 shifted by -rho."""
    if dense is not None:
        return dense - rho * np.eye(dense.shape[0])
    return dirac.dense_matrix(U, -rho)


def hermitian_kernel(dk):
    """H = gamma5 D_kn(-rho)."""
    g5 = gamma5_full(dk.shape[0] // 12)
    return g5 @ dk


def sign_matrix(h):
    """sign(H) = V sign(Lambda) V^dag for Hermitian H."""
    w, v = np.linalg.eigh(h)
    return (v * np.sign(w)[None, :]) @ v.conj().T


def overlap_matrix(dk, rho=RHO, mass=0.0):
    """D_ov,m of Eqs. def_over and def_mass from the shifted kernel dk = D_kn(-rho)."""
    n = dk.shape[0]
    g5 = gamma5_full(n // 12)
    dov = rho * (np.eye(n) + g5 @ sign_matrix(g5 @ dk))
    return (1.0 - mass / (2.0 * rho)) * dov + mass * np.eye(n)


def ritz_reference(dk):
    """Exact eigenvalues of A = D^dag D (ascending): what Ritz values approximate."""
    return np.linalg.eigvalsh(dk.conj().T @ dk)


def inv_sqrt_chebyshev(lo, hi, degree):
    """Coefficients c_0..c_N of the Chebyshev interpolant of x^{-1/2} on [lo, hi]
    in the variable t = (2x - hi - lo)/(hi - lo), from the N+1 Chebyshev-Gauss
    nodes, and the interpolant's maximum relative deviation |1 - sqrt(x) p(x)|
    on a fine grid."""
    n = degree + 1
    j = np.arange(n)
    t = np.cos(np.pi * (j + 0.5) / n)
    x = 0.5 * (hi - lo) * t + 0.5 * (hi + lo)
    f = 1.0 / np.sqrt(x)
    c = np.array([2.0 / n * np.sum(f * np.cos(np.pi * k * (j + 0.5) / n)) for k in range(n)])
    c[0] *= 0.5
    xs = np.linspace(lo, hi, 20001)
    ts = (2 * xs - hi - lo) / (hi - lo)
    p = np.polynomial.chebyshev.chebval(ts, c)
    return c, float(np.max(np.abs(1.0 - np.sqrt(xs) * p)))
