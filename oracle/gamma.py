"""Euclidean gamma matrices for the oracle.

The paper only requires a 4-dimensional Hermitian representation with
gamma5-hermiticity (Sec. 1; the 4D Dirac-Clifford algebra of Sec. 4).  The
representation adopted here is the chiral one built from the Pauli matrices:

    gamma_k = [[0, -i sigma_k], [i sigma_k, 0]]   (k = 1, 2, 3 -> mu = 0, 1, 2)
    gamma_4 = [[0, 1], [1, 0]]                     (mu = 3, the t direction)
    gamma_5 = gamma_1 gamma_2 gamma_3 gamma_4 = diag(1, 1, -1, -1)

Parity: pinned (Clifford algebra, hermiticity and gamma5 checked in tests;
every physics pin is basis independent).
"""
from __future__ import annotations

import numpy as np

SIGMA = [
    np.array([[0, 1], [1, 0]], dtype=np.complex128),
    np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    np.array([[1, 0], [0, -1]], dtype=np.complex128),
]
_Z = np.zeros((2, 2), dtype=np.complex128)
_I2 = np.eye(2, dtype=np.complex128)


def gammas():
    """List [gamma_x, gamma_y, gamma_z, gamma_t] of 4x4 complex matrices."""
    g = [np.block([[_Z, -1j * s], [1j * s, _Z]]) for s in SIGMA]
    g.append(np.block([[_Z, _I2], [_I2, _Z]]))
    return g


def gamma5():
    g = gammas()
    return g[0] @ g[1] @ g[2] @ g[3]
