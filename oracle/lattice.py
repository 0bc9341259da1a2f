"""Whole-lattice helpers for the oracle: periodic shifts and offsets.

Arrays are indexed [t, z, y, x, ...]; direction mu = 0, 1, 2, 3 is x, y, z, t,
so direction mu lives on array axis 3 - mu.  Boundary conditions are periodic
in all four directions (the paper does not state them; periodic is the
reading adopted for every lattice here).
"""
from __future__ import annotations

import itertools

import numpy as np


def shift(f, n):
    """Return g with g(x) = f(x + n) for an integer 4-vector n = (nx, ny, nz, nt)."""
    g = f
    for mu in range(4):
        if n[mu]:
            g = np.roll(g, -int(n[mu]), axis=3 - mu)
    return g


def dag(a):
    return np.conj(np.swapaxes(a, -1, -2))


def all_offsets():
    """The 80 non-zero offsets n in {-1,0,1}^4, ordered with n_x fastest."""
    out = []
    for nt, nz, ny, nx in itertools.product((-1, 0, 1), repeat=4):
        n = (nx, ny, nz, nt)
        if any(n):
            out.append(n)
    return out


def hops(n):
    """Number of non-zero components k = |n|_1 of an offset in {-1,0,1}^4."""
    return sum(1 for v in n if v)
