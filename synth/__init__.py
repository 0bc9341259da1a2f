"""Seeded synthetic inputs for the Brillouin-operator path and its oracle.

This module only draws random numbers and arranges them in the canonical
array layouts; it contains none of the operator's arithmetic.  Both the CPU
oracle (``oracle/``) and the GPU binding consume the arrays it returns.

Canonical layouts (numpy, C order, complex128):

* lattice extents ``dims = (Lx, Ly, Lz, Lt)``; arrays are indexed
  ``[t, z, y, x]`` so that x runs fastest, i.e. the linear site index is
  ``x + Lx*(y + Ly*(z + Lz*t))``;
* gauge links ``U[mu, t, z, y, x, a, b]`` with ``mu = 0..3`` for x, y, z, t;
  ``U[mu](x)`` is the 3x3 colour matrix on the link from x to x + mu-hat;
* colour-spinor fields ``psi[t, z, y, x, s, c]`` (spin s = 0..3, colour
  c = 0..2), optionally with a leading right-hand-side axis.

Link distribution (the paper uses thermalised quenched ensembles, which are
not available; these stand in for them): ``U = exp(i*eps*H)`` with H a
traceless Hermitian matrix built from a complex Gaussian G (independent
N(0,1) real and imaginary parts) as ``H = (G + G^dag)/2 - tr(.)/3``.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "lattice_shape", "volume", "gauge_links", "gauge_links_device", "unit_links", "gaussian_spinor",
    "point_sources", "random_su3_field", "gauge_transform_links",
    "gauge_transform_spinor", "plane_wave", "mean_plaquette_trace",
]

_CHUNK = 1 << 20  # matrices per eigendecomposition batch (bounds host memory)


def lattice_shape(dims):
    """Array shape ``(Lt, Lz, Ly, Lx)`` for extents ``dims = (Lx, Ly, Lz, Lt)``."""
    lx, ly, lz, lt = (int(v) for v in dims)
    return (lt, lz, ly, lx)


def volume(dims):
    return int(np.prod([int(v) for v in dims]))


def _complex_normal(rng, shape):
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return re + 1j * im


def _expi_traceless_hermitian(rng, n, eps):
    """n matrices exp(i*eps*H), H traceless Hermitian from a complex Gaussian."""
    out = np.empty((n, 3, 3), dtype=np.complex128)
    for lo in range(0, n, _CHUNK):
        hi = min(n, lo + _CHUNK)
        g = _complex_normal(rng, (hi - lo, 3, 3))
        h = 0.5 * (g + np.conj(np.swapaxes(g, -1, -2)))
        tr = np.trace(h, axis1=-2, axis2=-1).real / 3.0
        h -= tr[:, None, None] * np.eye(3)
        w, v = np.linalg.eigh(h)
        out[lo:hi] = (v * np.exp(1j * eps * w)[:, None, :]) @ np.conj(np.swapaxes(v, -1, -2))
    return out


def gauge_links(dims, eps, seed):
    """Random SU(3) links ``U[mu,t,z,y,x,3,3]`` = exp(i*eps*H), seeded."""
    rng = np.random.default_rng(seed)
    shp = lattice_shape(dims)
    n = 4 * volume(dims)
    return _expi_traceless_hermitian(rng, n, float(eps)).reshape((4,) + shp + (3, 3))


def gauge_links_device(dims, eps, seed, device="cuda"):
    """Same distribution as ``gauge_links`` drawn with torch's seeded generator
    on ``device`` (for lattices where the host eigendecompositions would take
    minutes).  U = exp(i eps H) by ``torch.linalg.matrix_exp``.  Returns a
    complex128 tensor [4, Lt, Lz, Ly, Lx, 3, 3]; not bit-identical to
    ``gauge_links`` for the same seed."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    shp = (4,) + lattice_shape(dims) + (3, 3)
    out = torch.empty(shp, dtype=torch.complex128, device=device)
    flat = out.view(-1, 3, 3)
    eye = torch.eye(3, dtype=torch.complex128, device=device)
    for lo in range(0, flat.shape[0], _CHUNK):
        hi = min(flat.shape[0], lo + _CHUNK)
        re = torch.randn((hi - lo, 3, 3), generator=gen, dtype=torch.float64, device=device)
        im = torch.randn((hi - lo, 3, 3), generator=gen, dtype=torch.float64, device=device)
        g = torch.complex(re, im)
        h = 0.5 * (g + g.conj().transpose(-1, -2))
        tr = torch.diagonal(h, dim1=-2, dim2=-1).sum(-1).real / 3.0
        h = h - tr[:, None, None] * eye
        flat[lo:hi] = torch.linalg.matrix_exp(1j * eps * h)
    return out


def unit_links(dims):
    shp = lattice_shape(dims)
    u = np.zeros((4,) + shp + (3, 3), dtype=np.complex128)
    u[..., 0, 0] = u[..., 1, 1] = u[..., 2, 2] = 1.0
    return u


def gaussian_spinor(dims, seed, nrhs=None):
    """Gaussian colour-spinor field (independent N(0,1) real/imag parts)."""
    rng = np.random.default_rng(seed)
    shp = lattice_shape(dims) + (4, 3)
    if nrhs is not None:
        shp = (int(nrhs),) + shp
    return _complex_normal(rng, shp)


def point_sources(dims, site=(0, 0, 0, 0)):
    """The 12 spin-colour point sources at ``site = (x, y, z, t)``:
    ``out[3*s + c]`` is the unit vector e_s (x) e_c at that site."""
    shp = lattice_shape(dims)
    out = np.zeros((12,) + shp + (4, 3), dtype=np.complex128)
    x, y, z, t = site
    for s in range(4):
        for c in range(3):
            out[3 * s + c, t, z, y, x, s, c] = 1.0
    return out


def random_su3_field(dims, seed):
    """Haar-random SU(3) matrices g[t,z,y,x,3,3] (QR of a complex Gaussian,
    phases fixed, determinant divided out)."""
    rng = np.random.default_rng(seed)
    shp = lattice_shape(dims)
    n = volume(dims)
    z = _complex_normal(rng, (n, 3, 3)) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=-2, axis2=-1)
    q = q * (d / np.abs(d))[:, None, :]
    det = np.linalg.det(q)
    q = q / (det ** (1.0 / 3.0))[:, None, None]
    return q.reshape(shp + (3, 3))


def _shift(f, mu, step):
    """f(x + step*mu-hat) as a whole-lattice array (periodic)."""
    axis = 3 - mu
    return np.roll(f, -step, axis=axis)


def gauge_transform_links(u, g):
    """U^g_mu(x) = g(x) U_mu(x) g(x+mu)^dag."""
    out = np.empty_like(u)
    for mu in range(4):
        gp = _shift(g, mu, +1)
        out[mu] = g @ u[mu] @ np.conj(np.swapaxes(gp, -1, -2))
    return out


def gauge_transform_spinor(psi, g):
    """(g psi)(x) = g(x) psi(x), acting on colour."""
    return np.einsum("...ab,...sb->...sa", g, psi)


def plane_wave(dims, mom, chi):
    """psi(x) = exp(i k.x) chi with k_mu = 2 pi mom_mu / L_mu; chi is (4,3)."""
    lx, ly, lz, lt = dims
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx),
                             indexing="ij")
    ph = 2 * np.pi * (mom[0] * x / lx + mom[1] * y / ly + mom[2] * z / lz + mom[3] * t / lt)
    return np.exp(1j * ph)[..., None, None] * np.asarray(chi)[None, None, None, None]


def mean_plaquette_trace(u):
    """Average of Re tr(U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag)/3, reported
    as context for a synthetic configuration."""
    acc, cnt = 0.0, 0
    dag = lambda a: np.conj(np.swapaxes(a, -1, -2))
    for mu in range(4):
        for nu in range(mu + 1, 4):
            p = u[mu] @ _shift(u[nu], mu, 1) @ dag(_shift(u[mu], nu, 1)) @ dag(u[nu])
            acc += np.trace(p, axis1=-2, axis2=-1).real.mean() / 3.0
            cnt += 1
    return acc / cnt
