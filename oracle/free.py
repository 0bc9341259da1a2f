"""Free-field (unit link) momentum-space forms of the Brillouin operator.

With U = 1 the operator is diagonal in momentum: D e^{ik.x} chi = Dhat(k) chi
e^{ik.x}, where from Eq. def_4Dbri and the isotropic derivative of App. C

    Dhat(k) = m + 2 - 2 prod_nu cos^2(k_nu/2) + i sum_mu gamma_mu s_mu(k),
    s_mu(k) = sin(k_mu) prod_{nu != mu} (cos k_nu + 2)/3.

Writing A(k) = m + 2 - 2 prod cos^2(k/2), the inverse follows from the
gamma-matrix identity used in Sec. 2.4 for the 2D dispersion relation:
Dhat^{-1} = (A - i sum gamma_mu s_mu) / (A^2 + sum_mu s_mu^2), and the
eigenvalues of Dhat are A +- i|s| (each twice in spin, three times in colour).

``fourier_sum`` evaluates sum_n C(n) e^{ik.n} over the 81 stencil points
directly, a brute-force cross-check of the closed form.
"""
from __future__ import annotations

import numpy as np

from .constants import operator_weights
from .dirac import coefficient_matrix
from .gamma import gammas
from .lattice import all_offsets


def a_of_k(k, mass):
    return mass + 2.0 - 2.0 * np.prod(np.cos(np.asarray(k) / 2.0) ** 2, axis=-1)


def s_of_k(k):
    k = np.asarray(k, dtype=float)
    out = []
    for mu in range(4):
        v = np.sin(k[..., mu])
        for nu in range(4):
            if nu != mu:
                v = v * (np.cos(k[..., nu]) + 2.0) / 3.0
        out.append(v)
    return np.stack(out, axis=-1)


def symbol(k, mass):
    """Closed-form 4x4 Dhat(k) for a single momentum k (4,)."""
    g = gammas()
    s = s_of_k(k)
    out = a_of_k(k, mass) * np.eye(4, dtype=np.complex128)
    for mu in range(4):
        out = out + 1j * s[mu] * g[mu]
    return out


def fourier_sum(k, mass):
    """sum_n C(n) exp(i k.n) over n in {-1,0,1}^4 (unit links)."""
    lam, rho = operator_weights(mass)
    out = lam[(0, 0, 0, 0)] * np.eye(4, dtype=np.complex128)
    for n in all_offsets():
        out = out + coefficient_matrix(lam, rho, n) * np.exp(1j * np.dot(k, n))
    return out


def eigenvalues(k, mass):
    a = a_of_k(k, mass)
    s = np.sqrt((s_of_k(k) ** 2).sum(axis=-1))
    return a + 1j * s, a - 1j * s


def propagator_solve(dims, b, mass):
    """x with D x = b for unit links, by FFT and the closed-form inverse
    (Dhat^{-1} = (A - i sum gamma s)/(A^2 + |s|^2)).  b: (Lt,Lz,Ly,Lx,4,3)."""
    lx, ly, lz, lt = dims
    g = gammas()
    bh = np.fft.fftn(b, axes=(0, 1, 2, 3))
    kt, kz, ky, kx = np.meshgrid(2 * np.pi * np.fft.fftfreq(lt), 2 * np.pi * np.fft.fftfreq(lz),
                                 2 * np.pi * np.fft.fftfreq(ly), 2 * np.pi * np.fft.fftfreq(lx),
                                 indexing="ij")
    k = np.stack([kx, ky, kz, kt], axis=-1)
    a = a_of_k(k, mass)
    s = s_of_k(k)
    den = a ** 2 + (s ** 2).sum(axis=-1)
    inv = a[..., None, None] * np.eye(4)
    for mu in range(4):
        inv = inv - 1j * s[..., mu, None, None] * g[mu]
    inv = inv / den[..., None, None]
    xh = np.einsum("...st,...tc->...sc", inv, bh)
    return np.fft.ifftn(xh, axes=(0, 1, 2, 3))
