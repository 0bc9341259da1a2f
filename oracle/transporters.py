"""Gauge transporters W(x, x+n) for the 80 off-site stencil points.

Sec. 5.1: the derivative and the Laplacian are made gauge covariant by
connecting x with x+n through all shortest lattice paths; there are k! of them
for a k-hop offset (2, 6 and 24 for the 2-, 3- and 4-hop points).  Each path is
the ordered product of link variables, U_mu(y) for a step y -> y+mu-hat and
U_mu(y-mu-hat)^dag for a step y -> y-mu-hat (the link orientation of the Wilson
operator, Sec. 1: U_mu(x) multiplies psi(x+mu-hat)).

Reading adopted where the paper is silent or ambiguous: the path products are
AVERAGED (divided by k!) and not back-projected to SU(3).  With unit links the
average is the identity, so the covariant operator reduces to the free stencil
of App. C, which fixes the normalisation.

The oracle enumerates every path explicitly (itertools.permutations); it uses
no recursion and no sharing of sub-paths.

Parity: pinned (unit links give W = 1, path counts, W(x+n,x) = W(x,x+n)^dag,
the 2-hop closed form, gauge covariance, and agreement with the independent
factorised formulation in ``oracle.factorized``).
"""
from __future__ import annotations

import itertools

import numpy as np

from .lattice import shift, dag


def whole_lattice(field, d):
    """Getter: field(x + d) at every site (periodic)."""
    return shift(field, d)


def make_site_getter(sites, dims):
    """Getter restricted to sampled sites.

    ``sites`` is an integer array (N, 4) of coordinates (x, y, z, t); the getter
    returns field(site + d) for each sampled site, shape (N, ...)."""
    sites = np.asarray(sites, dtype=np.int64)
    lx, ly, lz, lt = dims

    def get(field, d):
        x = (sites[:, 0] + d[0]) % lx
        y = (sites[:, 1] + d[1]) % ly
        z = (sites[:, 2] + d[2]) % lz
        t = (sites[:, 3] + d[3]) % lt
        return field[t, z, y, x]

    return get


def link_step(U, mu, s, get, d):
    """The factor for a step from y = x+d in direction s*mu-hat, evaluated at
    every site x: U_mu(y) for s = +1, U_mu(y - mu-hat)^dag for s = -1."""
    if s > 0:
        return get(U[mu], d)
    e = list(d)
    e[mu] -= 1
    return dag(get(U[mu], e))


def path_orderings(n):
    """All orderings of the directions in the support of n (k! of them)."""
    supp = [mu for mu in range(4) if n[mu]]
    return list(itertools.permutations(supp))


def path_product(U, n, order, get=whole_lattice):
    """Ordered link product along the path from x to x+n that steps through the
    directions in ``order`` (each once, with the sign of n_mu)."""
    d = [0, 0, 0, 0]
    prod = None
    for mu in order:
        a = link_step(U, mu, n[mu], get, d)
        prod = a if prod is None else prod @ a
        d[mu] += n[mu]
    return prod


def transporter(U, n, get=whole_lattice):
    """W(x, x+n): the average of the path products over all k! shortest paths."""
    orders = path_orderings(n)
    acc = None
    for order in orders:
        p = path_product(U, n, order, get)
        acc = p if acc is None else acc + p
    return acc / len(orders)


def all_transporters(U, offsets):
    """Dict n -> W(x, x+n) on the whole lattice (memory: 80 x V x 144 B)."""
    return {n: transporter(U, n) for n in offsets}


def two_hop_closed_form(U, mu, nu):
    """(U_mu(x) U_nu(x+mu) + U_nu(x) U_mu(x+nu)) / 2 for the (+mu, +nu) offset,
    written out as a pin for the general enumeration."""
    emu = [0, 0, 0, 0]
    emu[mu] = 1
    enu = [0, 0, 0, 0]
    enu[nu] = 1
    return 0.5 * (U[mu] @ shift(U[nu], emu) + U[nu] @ shift(U[mu], enu))


def max_spectral_norm(w):
    """Largest 2-norm over sites of a field of 3x3 matrices."""
    return float(np.linalg.norm(w.reshape(-1, 3, 3), ord=2, axis=(-2, -1)).max())
