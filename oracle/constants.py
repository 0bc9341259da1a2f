"""Stencil weights of the Brillouin operator, derived from momentum space.

The paper gives the 4D Brillouin Laplacian and the 4D isotropic derivative by
their momentum-space symbols (Sec. 4.1, Eq. def_4Dbri; App. C, isotropic
x-derivative):

    a^2 Lap^bri(k)  = 4 cos^2(k1/2) cos^2(k2/2) cos^2(k3/2) cos^2(k4/2) - 4
    a d^iso_1(k)    = i sin(k1) [cos(k2)+2][cos(k3)+2][cos(k4)+2] / 27

(the mu-derivative is the same with k_mu and k_1 exchanged).  A stencil with
support in {-1,0,1}^4 has symbol sum_n w(n) exp(i k.n), so w(n) is recovered
exactly by an inverse discrete Fourier transform of the symbol sampled on an
N^4 momentum grid with N >= 3.  That is what this module does; nothing here is
typed from the position-space tables, which the tests then use as pins
(App. C tables, Tab. rholambda).

Parity: pinned (App. C stencil tables, Tab. rholambda fractions, the
normalisation and doubler conditions of Sec. 8).
"""
from __future__ import annotations

from fractions import Fraction
import itertools

import numpy as np

from .lattice import all_offsets, hops

_NGRID = 6  # momentum grid points per direction for the inverse DFT (>= 3)


def lap_bri_symbol(k):
    """a^2 Lap^bri(k) for k of shape (..., 4) (Eq. def_4Dbri)."""
    return 4.0 * np.prod(np.cos(k / 2.0) ** 2, axis=-1) - 4.0


def der_iso_symbol(k, mu):
    """a d^iso_mu(k) (App. C, isotropic derivative, direction mu)."""
    out = 1j * np.sin(k[..., mu])
    for nu in range(4):
        if nu != mu:
            out = out * (np.cos(k[..., nu]) + 2.0)
    return out / 27.0


def _stencil_from_symbol(symbol):
    """Position-space weights w[n] (n in {-1,0,1}^4, indexed [nx+1,ny+1,nz+1,nt+1])
    from a momentum-space symbol sum_n w(n) e^{i k.n}, via inverse DFT."""
    n = _NGRID
    ks = 2 * np.pi * np.arange(n) / n
    kk = np.stack(np.meshgrid(ks, ks, ks, ks, indexing="ij"), axis=-1)  # [i0,i1,i2,i3,mu]
    s = symbol(kk)
    w = np.zeros((3, 3, 3, 3), dtype=np.complex128)
    for off in itertools.product((-1, 0, 1), repeat=4):
        ph = np.exp(-1j * (kk @ np.array(off, dtype=float)))
        w[tuple(o + 1 for o in off)] = (s * ph).sum() / n ** 4
    # anything outside {-1,0,1}^4 would alias; check the grid reproduces the symbol
    rec = np.zeros(kk.shape[:-1], dtype=np.complex128)
    for off in itertools.product((-1, 0, 1), repeat=4):
        rec += w[tuple(o + 1 for o in off)] * np.exp(1j * (kk @ np.array(off, dtype=float)))
    assert np.allclose(rec, s, atol=1e-12), "symbol is not supported on {-1,0,1}^4"
    return w


def laplacian_weights():
    """Real weights of a^2 Lap^bri, array [nx+1, ny+1, nz+1, nt+1]."""
    w = _stencil_from_symbol(lap_bri_symbol)
    assert np.abs(w.imag).max() < 1e-13
    return w.real.copy()


def derivative_weights():
    """Real weights of a d^iso_mu, array [mu, nx+1, ny+1, nz+1, nt+1]."""
    out = np.zeros((4, 3, 3, 3, 3))
    for mu in range(4):
        w = _stencil_from_symbol(lambda k, mu=mu: der_iso_symbol(k, mu))
        assert np.abs(w.imag).max() < 1e-13
        out[mu] = w.real
    return out


def as_fraction(x, max_den=100000):
    return Fraction(float(x)).limit_denominator(max_den)


def operator_weights(mass):
    """Per-offset coefficients of D = sum_mu gamma_mu d^iso_mu - Lap^bri/2 + m
    (Eq. def_pref with a = 1, c_SW = 0):

    returns (lam, rho) with lam[n] the identity coefficient and rho[n][mu] the
    gamma_mu coefficient, as dicts keyed by the offset tuple n (n = 0 included).
    """
    lap = laplacian_weights()
    der = derivative_weights()
    lam, rho = {}, {}
    for n in [(0, 0, 0, 0)] + all_offsets():
        idx = tuple(v + 1 for v in n)
        lam[n] = -0.5 * lap[idx] + (mass if not any(n) else 0.0)
        rho[n] = np.array([der[mu][idx] for mu in range(4)])
    return lam, rho


def class_coefficients():
    """(lambda_k, rho_k) for hop class k = 0..4 as exact fractions, read off the
    derived weights: lambda(n) = lambda_k, rho_mu(n) = rho_k * n_mu (the
    ultralocal form of Sec. 8, Tab. rholambda).  Raises if the derived
    weights do not have that class structure."""
    lam, rho = operator_weights(0.0)
    lam_k, rho_k = {}, {}
    for n in [(0, 0, 0, 0)] + all_offsets():
        k = hops(n)
        lf = as_fraction(lam[n])
        if k in lam_k:
            assert lam_k[k] == lf, (n, lf, lam_k[k])
        lam_k[k] = lf
        for mu in range(4):
            rf = as_fraction(rho[n][mu])
            if n[mu] == 0:
                assert rf == 0, (n, mu, rf)
            else:
                r = rf * n[mu]
                if k in rho_k:
                    assert rho_k[k] == r, (n, mu, r, rho_k[k])
                rho_k[k] = r
    return lam_k, rho_k
