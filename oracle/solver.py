"""Conjugate gradients on the normal equations (CGNE), FP64, for the oracle.

The paper inverts the Dirac operator with BiCGstab to a residual norm of 1e-7
(Sec. 6.4) and notes that the CG cost scales with sqrt(cond(D^dag D)).  The
solver here is plain CG on D^dag D x = D^dag b (textbook Hestenes-Stiefel),
stopped when the true relative residual ||b - D x|| / ||b|| is at most tol.

Parity: pinned (dense LU solve at 4^4; free-field FFT propagator).
"""
from __future__ import annotations

import numpy as np

from . import dirac


def _dot(a, b):
    return np.vdot(a, b)


def cgne(U, b, mass, tol=1e-10, max_iter=10000, x0=None, apply=None, apply_dag=None):
    """Solve D x = b.  Returns (x, iterations, true relative residual)."""
    apply = apply or (lambda f: dirac.apply(U, f, mass))
    apply_dag = apply_dag or (lambda f: dirac.apply_dag(U, f, mass))
    x = np.zeros_like(b) if x0 is None else x0.copy()
    bnorm = np.sqrt(_dot(b, b).real)
    r = b - apply(x) if x0 is not None else b.copy()
    z = apply_dag(r)        # residual of the normal equations
    p = z.copy()
    zz = _dot(z, z).real
    it = 0
    while it < max_iter:
        q = apply(p)
        alpha = zz / _dot(q, q).real
        x = x + alpha * p
        r = r - alpha * q
        it += 1
        if np.sqrt(_dot(r, r).real) <= tol * bnorm:
            true = b - apply(x)
            if np.sqrt(_dot(true, true).real) <= tol * bnorm:
                break
            r = true
        z = apply_dag(r)
        zz_new = _dot(z, z).real
        p = z + (zz_new / zz) * p
        zz = zz_new
    true = b - apply(x)
    return x, it, float(np.sqrt(_dot(true, true).real) / bnorm)
