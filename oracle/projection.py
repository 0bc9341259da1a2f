"""Projection of a 3x3 complex matrix to U(3) and to SU(3) (Sec. 5.2).

TEST INFRASTRUCTURE ONLY (see the package docstring).

* ``project_un``: Eq. def_projection, P_U(N){A} = A (A^dag A)^{-1/2} = U V^dag
  for the singular value decomposition A = U S V^dag.
* ``project_sun``: Eq. proj_SU, the SU(N) element closest to A in the
  Frobenius norm, by the three steps of Sec. 5.2:
    1. A = U S V^dag (numpy's SVD);
    2. det(U V^dag) = exp(i phi);
    3. phases D = diag(exp(i theta_j)) with sum_j theta_j + phi = 0 (mod 2 pi)
       that maximise Re tr(A^dag U D V^dag) = sum_j s_j cos(theta_j); the
       global maximum is located by a scan of (theta_1, theta_2) over a grid
       of spacing pi/3 (the paper's suggestion, 6^(N-1) = 36 points),
       followed by a local maximisation (Newton's method with a backtracking
       line search) from the best grid point;
  and Y = U D V^dag.

Both act on arrays of shape (..., 3, 3).

Parity: pinned (unitarity and unit determinant of the result, SU(3) inputs
returned unchanged, invariance under positive rescaling, covariance under
A -> g1 A g2^dag, the closed form for a multiple of a U(3) matrix, the
diagonal U(1)-embedding case, and global optimality against a fine brute
force scan of the two free phases and against random SU(3) samples).
"""
from __future__ import annotations

import numpy as np

N = 3
_SCAN = np.arange(6) * (np.pi / 3.0)


def _dag(a):
    return np.conj(np.swapaxes(a, -1, -2))


def project_un(a):
    """P_U(3){A} = U V^dag (Eq. def_projection)."""
    u, _, vh = np.linalg.svd(a)
    return u @ vh


def objective(s, phi, th1, th2):
    """sum_j s_j cos(theta_j) with theta_3 = -phi - theta_1 - theta_2."""
    th3 = -phi - th1 - th2
    return s[..., 0] * np.cos(th1) + s[..., 1] * np.cos(th2) + s[..., 2] * np.cos(th3)


def maximise_phases(s, phi, iters=100):
    """The constrained phase maximisation of step 3 for a batch.

    s: (M, 3) singular values, phi: (M,).  Returns theta (M, 3)."""
    s = np.asarray(s, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    m = s.shape[0]
    # coarse scan over the grid of spacing pi/3
    g1, g2 = np.meshgrid(_SCAN, _SCAN, indexing="ij")
    g1 = g1.reshape(-1)
    g2 = g2.reshape(-1)
    f = objective(s[:, None, :], phi[:, None], g1[None, :], g2[None, :])
    best = np.argmax(f, axis=1)
    t1 = g1[best].copy()
    t2 = g2[best].copy()
    # local maximisation: Newton steps on (theta_1, theta_2); a gradient step
    # replaces Newton's where the Hessian is not negative definite.  Steps
    # longer than 0.5 (or gradient steps) are halved until the objective does
    # not decrease; short Newton steps are taken whole, since near the
    # maximum the gain in the objective falls below its rounding error
    for _ in range(iters):
        t3 = -phi - t1 - t2
        sn1, sn2, sn3 = np.sin(t1), np.sin(t2), np.sin(t3)
        c1, c2, c3 = np.cos(t1), np.cos(t2), np.cos(t3)
        gr1 = -s[:, 0] * sn1 + s[:, 2] * sn3
        gr2 = -s[:, 1] * sn2 + s[:, 2] * sn3
        if np.all(np.abs(gr1) + np.abs(gr2) <= 1e-15 * s.sum(axis=1)):
            break
        h11 = -s[:, 0] * c1 - s[:, 2] * c3
        h22 = -s[:, 1] * c2 - s[:, 2] * c3
        h12 = -s[:, 2] * c3
        det = h11 * h22 - h12 * h12
        negdef = (h11 < 0) & (det > 0)
        safe = np.where(negdef, det, 1.0)
        d1 = np.where(negdef, -(h22 * gr1 - h12 * gr2) / safe, gr1 / (2.0 * s.sum(axis=1)))
        d2 = np.where(negdef, -(-h12 * gr1 + h11 * gr2) / safe, gr2 / (2.0 * s.sum(axis=1)))
        short = negdef & (np.maximum(np.abs(d1), np.abs(d2)) <= 0.5)
        f0 = objective(s, phi, t1, t2)
        step = np.ones(m)
        for _ in range(60):
            f1 = objective(s, phi, t1 + step * d1, t2 + step * d2)
            bad = (f1 < f0) & ~short
            if not bad.any():
                break
            step = np.where(bad, 0.5 * step, step)
        ok = short | (objective(s, phi, t1 + step * d1, t2 + step * d2) >= f0)
        t1 = np.where(ok, t1 + step * d1, t1)
        t2 = np.where(ok, t2 + step * d2, t2)
    return np.stack([t1, t2, -phi - t1 - t2], axis=1)


def project_sun(a):
    """P_SU(3){A}: the closest SU(3) matrix (Eq. proj_SU, Sec. 5.2)."""
    a = np.asarray(a, dtype=np.complex128)
    shape = a.shape
    flat = a.reshape(-1, N, N)
    u, s, vh = np.linalg.svd(flat)
    phi = np.angle(np.linalg.det(u) * np.linalg.det(vh))
    theta = maximise_phases(s, phi)
    y = (u * np.exp(1j * theta)[:, None, :]) @ vh
    return y.reshape(shape)


def naive_sun(a):
    """U V^dag divided by the cube root of its determinant (the recipe the
    paper rejects); used only to compare distances in the tests."""
    x = project_un(a)
    d = np.linalg.det(x)
    return x / (d ** (1.0 / N))[..., None, None]


def distance2(a, y):
    """tr (A - Y)^dag (A - Y) per matrix."""
    e = a - y
    return np.real(np.einsum("...ab,...ab->...", np.conj(e), e))
