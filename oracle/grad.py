"""Gradients of S = Re <chi, D psi> = Re sum_x chi(x)^dag (D psi)(x).

Complex gradients use the convention g = dS/dRe(z) + i dS/dIm(z) (the one
PyTorch uses for real losses of complex tensors).  Link entries are treated
as unconstrained complex numbers.

* psi:   g_psi = D^dag chi.
* links: each offset contributes Re sum_x tr[W(x,x+n) K_n(x)] with
  K_n(x) = sum_s psi_s(x+n) (C(n)^dag chi(x))_s^dag, so the transporter
  receives G_W(x,n) = K_n(x)^dag = sum_s (C(n)^dag chi(x))_s psi_s(x+n)^dag.
  W is the average of path products A_1 ... A_k (Sec. 5.1), and the chain rule
  for a product gives G_{A_j} = (A_1..A_{j-1})^dag G_W (A_{j+1}..A_k)^dag / k!.
  A forward step A_j = U_mu(y) passes G_{A_j} to U_mu(y); a backward step
  A_j = U_mu(y - mu-hat)^dag passes G_{A_j}^dag to U_mu(y - mu-hat).

Every path is enumerated explicitly; no recursion is shared with the GPU
library.

For S2 = phi^dag (D^dag D)^{-1} phi with X = (D^dag D)^{-1} phi the first
variation is dS2 = -2 Re <D X, dD X>, so dS2/dU is the link gradient above with
(chi, psi) = (-2 D X, X), and dS2/dphi = 2 X.

``table`` (optional) takes another member of the generic class of Sec. 8
(``oracle.ultralocal``); S then uses that operator.

Parity: pinned (central finite differences of the oracle's own S, which is
itself pinned, for the Brillouin operator and for a generic-class table;
closed-form psi gradient).
"""
from __future__ import annotations

import numpy as np

from .constants import operator_weights
from .dirac import coefficient_matrix, apply_dag
from .lattice import all_offsets, shift, dag
from .transporters import link_step, path_orderings, whole_lattice


def action(U, chi, psi, mass, table=None):
    from .dirac import apply
    from . import ultralocal
    d = apply(U, psi, mass) if table is None else ultralocal.apply(U, psi, mass, table)
    return float(np.vdot(chi, d).real)


def grad_psi(U, chi, mass, table=None):
    from . import ultralocal
    return apply_dag(U, chi, mass) if table is None else ultralocal.apply_dag(U, chi, mass, table)


def grad_links(U, chi, psi, mass, table=None):
    """dS/dU for S = Re <chi, D psi>; same shape as U."""
    from . import ultralocal
    lam, rho = operator_weights(mass) if table is None else ultralocal.weights(table, mass)
    gu = np.zeros_like(U)
    for n in all_offsets():
        phi = np.einsum("ts,...tc->...sc", np.conj(coefficient_matrix(lam, rho, n)), chi)  # C^dag chi
        gw = np.einsum("...sa,...sb->...ab", phi, np.conj(shift(psi, n)))
        orders = path_orderings(n)
        for order in orders:
            factors, disp = [], []
            d = [0, 0, 0, 0]
            for mu in order:
                factors.append(link_step(U, mu, n[mu], whole_lattice, d))
                disp.append(list(d))
                d[mu] += n[mu]
            k = len(factors)
            for j in range(k):
                left = None
                for a in factors[:j]:
                    left = a if left is None else left @ a
                right = None
                for a in factors[j + 1:]:
                    right = a if right is None else right @ a
                g = gw
                if left is not None:
                    g = dag(left) @ g
                if right is not None:
                    g = g @ dag(right)
                g = g / len(orders)
                mu = order[j]
                dj = disp[j]
                if n[mu] > 0:
                    gu[mu] += shift(g, [-v for v in dj])
                else:
                    base = list(dj)
                    base[mu] -= 1
                    gu[mu] += shift(dag(g), [-v for v in base])
    return gu
