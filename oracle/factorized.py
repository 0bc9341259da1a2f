"""Second, independent formulation of the Brillouin operator (used as a pin).

Both momentum-space symbols are products of one-dimensional factors
(Eq. def_4Dbri; App. C isotropic derivative; App. D factorises the isotropic
stencils the same way):

    4 prod_mu cos^2(k_mu/2) = prod_mu (2 + 2 cos k_mu) / 64
    i sin(k_mu) prod_{nu!=mu} (cos k_nu + 2)/27
        = [(e^{ik_mu} - e^{-ik_mu})/2] prod_{nu!=mu} (4 + 2 cos k_nu)/6

With the covariant one-step hops H+_mu psi(x) = U_mu(x) psi(x+mu-hat) and
H-_mu psi(x) = U_mu(x-mu-hat)^dag psi(x-mu-hat), replace 2 cos k_mu by
H+_mu + H-_mu and i sin k_mu by (H+_mu - H-_mu)/2.  A product of such hop
operators in a fixed order transports along one path; averaging the product
over all orderings of the four factors gives every shortest path to x+n the
same weight 1/k!, i.e. the path-averaged transporter of Sec. 5.1.  So

    Lap^bri       = [ avg_sigma S_s1 S_s2 S_s3 S_s4 - 256 ] / 64,
                    S_mu = 2 + H+_mu + H-_mu,
    d^iso_mu      = avg over orderings of { (H+_mu - H-_mu)/2, T_nu/6 (nu != mu) },
                    T_nu = 4 + H+_nu + H-_nu,

and the ordering average is evaluated by the subset recursion
P_A = (1/|A|) sum_{mu in A} O_mu P_{A \\ mu}, P_{} = psi.

This code shares nothing with ``oracle.transporters`` (no path enumeration, no
transporter matrices): agreement of the two to rounding pins both.
"""
from __future__ import annotations

from itertools import combinations

import numpy as np

from .gamma import gammas
from .lattice import shift, dag


def _hop_plus(U, mu, psi):
    e = [0, 0, 0, 0]
    e[mu] = 1
    return np.einsum("...ab,...sb->...sa", U[mu], shift(psi, e))


def _hop_minus(U, mu, psi):
    e = [0, 0, 0, 0]
    e[mu] = -1
    return np.einsum("...ab,...sb->...sa", dag(shift(U[mu], e)), shift(psi, e))


def _ordering_average(ops, psi):
    """avg over all orderings of the product ops[s1] ops[s2] ops[s3] ops[s4] psi."""
    p = {(): psi}
    for size in range(1, len(ops) + 1):
        for a in combinations(range(len(ops)), size):
            acc = None
            for mu in a:
                rest = tuple(v for v in a if v != mu)
                term = ops[mu](p[rest])
                acc = term if acc is None else acc + term
            p[a] = acc / size
    return p[tuple(range(len(ops)))]


def laplacian(U, psi):
    """Lap^bri psi."""
    ops = [lambda f, mu=mu: 2.0 * f + _hop_plus(U, mu, f) + _hop_minus(U, mu, f)
           for mu in range(4)]
    return (_ordering_average(ops, psi) - 256.0 * psi) / 64.0


def derivative(U, psi, mu):
    """d^iso_mu psi."""
    ops = []
    for nu in range(4):
        if nu == mu:
            ops.append(lambda f, nu=nu: 0.5 * (_hop_plus(U, nu, f) - _hop_minus(U, nu, f)))
        else:
            ops.append(lambda f, nu=nu: (4.0 * f + _hop_plus(U, nu, f) + _hop_minus(U, nu, f)) / 6.0)
    return _ordering_average(ops, psi)


def apply(U, psi, mass):
    """D psi = sum_mu gamma_mu d^iso_mu psi - Lap^bri psi / 2 + m psi."""
    g = gammas()
    out = mass * psi - 0.5 * laplacian(U, psi)
    for mu in range(4):
        out = out + np.einsum("st,...tc->...sc", g[mu], derivative(U, psi, mu))
    return out
