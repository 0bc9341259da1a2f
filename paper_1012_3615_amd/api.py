"""Python binding of the C ABI (include/bri.h): argument marshalling only.

Every function forwards to the library entry point of the same name; torch
tensors supply device memory and the current HIP stream.  SoA buffers are
real tensors whose last axis holds (re, im):

    spinors       [nrhs, 12, V, 2]     component = 3*spin + colour
    links         [4, 9, V, 2]         element   = 3*a + b
    transporters  [n_offsets, 9, V, 2]   (two-row SU(3) form: [n_offsets, 6, V, 2])
    matrix-core transporter store  [V, 80, 9, 2] float16 (site-major)
    site-major spinors (matrix-core apply)  [V, nrhs, 12, 2] float32
    clover term   [2, 18, V, 2]

with dtype float64 (F64), float32 (F32) or float16 (F16).  Canonical fields
are complex128 tensors [4, Lt, Lz, Ly, Lx, 3, 3] (links) and
[nrhs, Lt, Lz, Ly, Lx, 4, 3] (spinors).
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib

F64, F32, F16 = 0, 1, 2
STORED, RECOMPUTE = 0, 1
W_AVERAGE, W_SU3, W_SU3_2ROW = 0, 1, 2

_lib_handle = _lib.load()

_TORCH = {F64: torch.float64, F32: torch.float32, F16: torch.float16}
_PREC = {torch.float64: F64, torch.float32: F32, torch.float16: F16}


class BriError(RuntimeError):
    def __init__(self, status, where):
        msg = _lib_handle.bri_last_error().decode(errors="replace")
        super().__init__(f"{where} failed with status {status}: {msg}")
        self.status = status


def lib():
    return _lib_handle


def _check(status, where):
    if status != 0:
        raise BriError(status, where)


def _dims(dims):
    d = _lib.bri_dims()
    for mu in range(4):
        d.L[mu] = int(dims[mu])
    return d


def volume(dims):
    v = 1
    for x in dims:
        v *= int(x)
    return v


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def prec_of(t):
    return _PREC[t.dtype]


def _need_cuda(*ts):
    for t in ts:
        if t is not None and (not t.is_cuda or not t.is_contiguous()):
            raise ValueError("expected contiguous device tensors")


# ------------------------------------------------------------------ allocation
def spinor_empty(dims, prec, nrhs=1, device="cuda"):
    return torch.empty((nrhs, 12, volume(dims), 2), dtype=_TORCH[prec], device=device)


def links_empty(dims, prec, device="cuda"):
    return torch.empty((4, 9, volume(dims), 2), dtype=_TORCH[prec], device=device)


def transporters_empty(dims, prec, n_offsets, device="cuda"):
    return torch.empty((n_offsets, 9, volume(dims), 2), dtype=_TORCH[prec], device=device)


# ------------------------------------------------------------------ layout
def bri_pack_links(dims, U_canon, prec=F64):
    _need_cuda(U_canon)
    if U_canon.dtype != torch.complex128 or U_canon.numel() != 36 * volume(dims):
        raise ValueError("links: expected complex128 [4, Lt, Lz, Ly, Lx, 3, 3]")
    out = links_empty(dims, prec, U_canon.device)
    _check(_lib_handle.bri_pack_links(_dims(dims), _ptr(U_canon), _ptr(out), prec, _stream()),
           "bri_pack_links")
    return out


def bri_pack_spinor(dims, psi_canon, prec=F64):
    _need_cuda(psi_canon)
    nrhs = psi_canon.numel() // (12 * volume(dims))
    if psi_canon.dtype != torch.complex128 or nrhs < 1 or psi_canon.numel() != 12 * volume(dims) * nrhs:
        raise ValueError("spinor: expected complex128 [nrhs, Lt, Lz, Ly, Lx, 4, 3]")
    out = spinor_empty(dims, prec, nrhs, psi_canon.device)
    _check(_lib_handle.bri_pack_spinor(_dims(dims), nrhs, _ptr(psi_canon), _ptr(out), prec,
                                       _stream()), "bri_pack_spinor")
    return out


def bri_unpack_spinor(dims, soa):
    _need_cuda(soa)
    _shape(soa, (soa.shape[0], 12, volume(dims), 2), "spinor")
    nrhs = soa.shape[0]
    lx, ly, lz, lt = dims
    out = torch.empty((nrhs, lt, lz, ly, lx, 4, 3), dtype=torch.complex128, device=soa.device)
    _check(_lib_handle.bri_unpack_spinor(_dims(dims), nrhs, _ptr(soa), prec_of(soa), _ptr(out),
                                         _stream()), "bri_unpack_spinor")
    return out


def bri_unpack_links(dims, soa):
    _need_cuda(soa)
    _shape(soa, (4, 9, volume(dims), 2), "links")
    lx, ly, lz, lt = dims
    out = torch.empty((4, lt, lz, ly, lx, 3, 3), dtype=torch.complex128, device=soa.device)
    _check(_lib_handle.bri_unpack_links(_dims(dims), _ptr(soa), prec_of(soa), _ptr(out), _stream()),
           "bri_unpack_links")
    return out


# ------------------------------------------------------------------ transporters
def bri_build_transporters(dims, U_soa, prec=F64, n_offsets=80, out=None):
    _need_cuda(U_soa)
    if prec_of(U_soa) != F64:
        raise ValueError("transporters are built from FP64 links")
    _shape(U_soa, (4, 9, volume(dims), 2), "links")
    if out is not None:
        _shape(out, (n_offsets, 9, volume(dims), 2), "transporters")
    W = out if out is not None else transporters_empty(dims, prec, n_offsets, U_soa.device)
    nbytes = _lib_handle.bri_build_workspace_bytes(_dims(dims), prec, n_offsets)
    work = torch.empty(max(nbytes, 16), dtype=torch.uint8, device=U_soa.device) if nbytes else None
    _check(_lib_handle.bri_build_transporters(_dims(dims), _ptr(U_soa), _ptr(W), prec, n_offsets,
                                              _ptr(work), nbytes, _stream()),
           "bri_build_transporters")
    return W


# ------------------------------------------------------------------ apply
def _shape(t, shape, what):
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{what}: expected shape {tuple(shape)}, got {tuple(t.shape)}")


def _apply(fn, name, dims, W_or_U, psi, mass, variant, out):
    _need_cuda(W_or_U, psi, out)
    V = volume(dims)
    _shape(psi, (psi.shape[0], 12, V, 2), "spinor")
    if variant == STORED:
        _shape(W_or_U, (W_or_U.shape[0], 9, V, 2), "transporters")
    else:
        _shape(W_or_U, (4, 9, V, 2), "links")
    if out is None:
        out = torch.empty_like(psi)
    elif out.shape != psi.shape or out.dtype != psi.dtype:
        raise ValueError("out must match the input spinor's shape and dtype")
    n_off = W_or_U.shape[0] if variant == STORED else 80
    _check(fn(_dims(dims), variant, _ptr(W_or_U), prec_of(W_or_U), n_off, prec_of(psi),
              float(mass), _ptr(psi), _ptr(out), psi.shape[0], _stream()), name)
    return out


def bri_apply(dims, W_or_U, psi, mass, variant=STORED, out=None):
    """out = D psi.  W_or_U: transporters (STORED) or SoA links (RECOMPUTE)."""
    return _apply(_lib_handle.bri_apply, "bri_apply", dims, W_or_U, psi, mass, variant, out)


def bri_apply_dag(dims, W_or_U, psi, mass, variant=STORED, out=None):
    """out = D^dag psi."""
    return _apply(_lib_handle.bri_apply_dag, "bri_apply_dag", dims, W_or_U, psi, mass, variant, out)


def bri_apply_wilson(dims, U, psi, mass, dagger=False, out=None):
    """out = D_W psi (or D_W^dag psi), the Wilson operator straight from the
    SoA links U; U and psi in the same precision (F64 or F32)."""
    _need_cuda(U, psi, out)
    V = volume(dims)
    _shape(psi, (psi.shape[0], 12, V, 2), "spinor")
    _shape(U, (4, 9, V, 2), "links")
    if U.dtype != psi.dtype:
        raise ValueError("links and spinor must have the same precision")
    if out is None:
        out = torch.empty_like(psi)
    elif out.shape != psi.shape or out.dtype != psi.dtype:
        raise ValueError("out must match the input spinor's shape and dtype")
    _check(_lib_handle.bri_apply_wilson(_dims(dims), _ptr(U), prec_of(U), float(mass), _ptr(psi), _ptr(out),
                                        psi.shape[0], int(bool(dagger)), _stream()), "bri_apply_wilson")
    return out


def _coef_arg(coef):
    if coef is None:
        return None, None
    coef = tuple(float(c) for c in coef)
    if len(coef) != 9:
        raise ValueError("a coefficient table has nine entries (lambda_0..4, rho_1..4)")
    arr = (ctypes.c_double * 9)(*coef)
    return arr, ctypes.addressof(arr)


def bri_pack_w_mfma(dims, W, out=None):
    """The site-major FP16 transporter store of the matrix-core apply
    ([V, 80, 9, 2] float16) from a 40- or 80-offset store W of any precision."""
    _need_cuda(W, out)
    V = volume(dims)
    _shape(W, (W.shape[0], 9, V, 2), "transporters")
    if out is None:
        out = torch.empty((V, 80, 9, 2), dtype=torch.float16, device=W.device)
    _shape(out, (V, 80, 9, 2), "matrix-core store")
    if out.dtype != torch.float16:
        raise ValueError("the matrix-core store is float16")
    _check(_lib_handle.bri_pack_w_mfma(_dims(dims), _ptr(W), prec_of(W), W.shape[0], _ptr(out), _stream()),
           "bri_pack_w_mfma")
    return out


def bri_spinor_bound2(dims, psi, out=None):
    """Per right-hand side the square of the largest |real or imaginary part|
    of an FP32 spinor field (float64 tensor [nrhs])."""
    _need_cuda(psi, out)
    _shape(psi, (psi.shape[0], 12, volume(dims), 2), "spinor")
    if psi.dtype != torch.float32:
        raise ValueError("bri_spinor_bound2 takes an FP32 field")
    if out is None:
        out = torch.empty(psi.shape[0], dtype=torch.float64, device=psi.device)
    _check(_lib_handle.bri_spinor_bound2(_dims(dims), psi.shape[0], _ptr(psi), _ptr(out), _stream()),
           "bri_spinor_bound2")
    return out


def bri_spinor_to_sites(dims, psi, out=None, bound2=None):
    """SoA FP32 spinor [nrhs, 12, V, 2] -> site-major [V, nrhs, 12, 2] (the
    layout of the matrix-core apply); with a float64 tensor bound2 [nrhs]
    (or True) also the per-right-hand-side bounds.  Returns the site-major
    field, or (field, bound2) when bounds were asked for."""
    _need_cuda(psi, out)
    V = volume(dims)
    _shape(psi, (psi.shape[0], 12, V, 2), "spinor")
    nrhs = psi.shape[0]
    if psi.dtype != torch.float32:
        raise ValueError("site-major fields are FP32")
    if out is None:
        out = torch.empty((V, nrhs, 12, 2), dtype=torch.float32, device=psi.device)
    _shape(out, (V, nrhs, 12, 2), "site-major spinor")
    want = bound2 is not None and bound2 is not False
    if bound2 is True:
        bound2 = torch.empty(nrhs, dtype=torch.float64, device=psi.device)
    _check(_lib_handle.bri_spinor_to_sites(_dims(dims), nrhs, _ptr(psi), _ptr(out), _ptr(bound2) if want else None,
                                           _stream()), "bri_spinor_to_sites")
    return (out, bound2) if want else out


def bri_spinor_from_sites(dims, psi_sites, out=None):
    """Site-major [V, nrhs, 12, 2] -> SoA [nrhs, 12, V, 2] (FP32)."""
    _need_cuda(psi_sites, out)
    V = volume(dims)
    nrhs = psi_sites.shape[1]
    _shape(psi_sites, (V, nrhs, 12, 2), "site-major spinor")
    if out is None:
        out = torch.empty((nrhs, 12, V, 2), dtype=torch.float32, device=psi_sites.device)
    _shape(out, (nrhs, 12, V, 2), "spinor")
    _check(_lib_handle.bri_spinor_from_sites(_dims(dims), nrhs, _ptr(psi_sites), _ptr(out), _stream()),
           "bri_spinor_from_sites")
    return out


def bri_apply_mfma(dims, Wm, psi_sites, mass, dagger=False, coef=None, bound2=None, out=None):
    """out = D psi (or D^dag psi) on the matrix cores: Wm from bri_pack_w_mfma,
    psi_sites and out site-major FP32 [V, nrhs, 12, 2] (bri_spinor_to_sites);
    bound2 (float64 [nrhs], device) bounds the squared components of psi, as
    bri_spinor_to_sites gives it; required."""
    _need_cuda(Wm, psi_sites, out, bound2)
    V = volume(dims)
    nrhs = psi_sites.shape[1]
    _shape(Wm, (V, 80, 9, 2), "matrix-core store")
    _shape(psi_sites, (V, nrhs, 12, 2), "site-major spinor")
    if psi_sites.dtype != torch.float32 or Wm.dtype != torch.float16:
        raise ValueError("the matrix-core apply takes an FP16 store and FP32 fields")
    if bound2 is None:
        raise ValueError("bound2 is required (bri_spinor_to_sites(..., bound2=True) gives it)")
    _shape(bound2, (nrhs,), "bound2")
    if out is None:
        out = torch.empty_like(psi_sites)
    elif out.shape != psi_sites.shape or out.dtype != psi_sites.dtype:
        raise ValueError("out must match the input spinor's shape and dtype")
    _keep, cptr = _coef_arg(coef)
    _check(_lib_handle.bri_apply_mfma(_dims(dims), _ptr(Wm), float(mass), _ptr(psi_sites), _ptr(out), nrhs,
                                      int(bool(dagger)), cptr, _ptr(bound2), _stream()), "bri_apply_mfma")
    return out


def bri_set_apply_config(dims, w_prec, s_prec, n_offsets, nrhs, kernel, rhs_per_thread=2):
    """Install (kernel, rhs_per_thread) for applies of exactly this shape;
    kernel = -1 removes the entry (the shape returns to the built-in choice)."""
    _check(_lib_handle.bri_set_apply_config(_dims(dims), w_prec, s_prec, n_offsets, nrhs, kernel,
                                            rhs_per_thread), "bri_set_apply_config")


def bri_get_apply_config(dims, w_prec, s_prec, n_offsets, nrhs):
    """(kernel code, right-hand sides per thread) that an apply of this shape
    launches (the built-in code 1 resolved to its tile)."""
    k, r = ctypes.c_int32(), ctypes.c_int32()
    _check(_lib_handle.bri_get_apply_config(_dims(dims), w_prec, s_prec, n_offsets, nrhs, ctypes.byref(k),
                                            ctypes.byref(r)), "bri_get_apply_config")
    return k.value, r.value


def bri_clear_apply_configs():
    _lib_handle.bri_clear_apply_configs()


# ------------------------------------------------------------------ solver
def solve_params(tol=1e-10, inner_tol=1e-4, max_iter=20000, max_outer=100, n_offsets=80,
                 inner_prec=F64, check_every=8, use_initial_guess=False, dagger=False, inner_mfma=False):
    """inner_mfma: inner applies on the matrix cores (inner_prec F16, W_lo
    from bri_pack_w_mfma)."""
    p = _lib.bri_solve_params()
    p.inner_mfma = int(bool(inner_mfma))
    p.tol, p.inner_tol = tol, inner_tol
    p.max_iter, p.max_outer = max_iter, max_outer
    p.n_offsets, p.inner_prec = n_offsets, inner_prec
    p.check_every, p.use_initial_guess = check_every, int(bool(use_initial_guess))
    p.dagger = int(bool(dagger))
    return p


def _solve_info(stats, nrhs, st):
    return {
        "iterations": stats.iterations, "outer": stats.outer, "applies": stats.applies,
        "converged": bool(stats.converged),
        "true_residual": [stats.true_residual[i] for i in range(min(nrhs, _lib.BRI_MAX_RHS))],
        "status": st,
    }


def _solve_args(dims, W_hi, b, params, W_lo, x):
    _need_cuda(W_hi, b, W_lo, x)
    V = volume(dims)
    _shape(b, (b.shape[0], 12, V, 2), "b")
    _shape(W_hi, (params.n_offsets, 9, V, 2), "W_hi")
    if W_lo is not None:
        _shape(W_lo, (V, 80, 9, 2) if params.inner_mfma else (params.n_offsets, 9, V, 2), "W_lo")
    if x is not None:
        _shape(x, b.shape, "x")
    if prec_of(b) != F64 or prec_of(W_hi) != F64:
        raise ValueError("b and W_hi must be FP64")
    if params.inner_prec != F64 and (W_lo is None or prec_of(W_lo) != params.inner_prec):
        raise ValueError("W_lo must be given in the inner precision")
    return x if x is not None else torch.zeros_like(b)


def bri_solve_cgne_noalloc(dims, W_hi, b, mass, params, W_lo=None, x=None, raise_on_noconv=True):
    """bri_solve_cgne without a workspace: the library's static per-device
    array serves as workspace (nothing is allocated except x when not given).
    Returns (x, stats dict)."""
    x = _solve_args(dims, W_hi, b, params, W_lo, x)
    nrhs = b.shape[0]
    stats = _lib.bri_solve_stats()
    st = _lib_handle.bri_solve_cgne_noalloc(_dims(dims), ctypes.byref(params), _ptr(W_hi), _ptr(W_lo),
                                            float(mass), _ptr(b), _ptr(x), nrhs, ctypes.byref(stats),
                                            _stream())
    info = _solve_info(stats, nrhs, st)
    if st != 0 and (raise_on_noconv or st != -4):
        raise BriError(st, "bri_solve_cgne_noalloc")
    return x, info


def bri_solve_cgne(dims, W_hi, b, mass, params, W_lo=None, x=None, raise_on_noconv=True):
    """Solve D x = b (or D^dag x = b with params.dagger) for FP64 SoA spinors.
    Returns (x, stats dict)."""
    _need_cuda(W_hi, b, W_lo, x)
    V = volume(dims)
    _shape(b, (b.shape[0], 12, V, 2), "b")
    _shape(W_hi, (params.n_offsets, 9, V, 2), "W_hi")
    if W_lo is not None:
        _shape(W_lo, (V, 80, 9, 2) if params.inner_mfma else (params.n_offsets, 9, V, 2), "W_lo")
    if x is not None:
        _shape(x, b.shape, "x")
    if prec_of(b) != F64 or prec_of(W_hi) != F64:
        raise ValueError("b and W_hi must be FP64")
    if params.inner_prec != F64 and (W_lo is None or prec_of(W_lo) != params.inner_prec):
        raise ValueError("W_lo must be given in the inner precision")
    nrhs = b.shape[0]
    if x is None:
        x = torch.zeros_like(b)
    nbytes = _lib_handle.bri_solve_workspace_bytes(_dims(dims), ctypes.byref(params), nrhs)
    work = torch.empty(max(nbytes, 16), dtype=torch.uint8, device=b.device)
    stats = _lib.bri_solve_stats()
    st = _lib_handle.bri_solve_cgne(_dims(dims), ctypes.byref(params), _ptr(W_hi), _ptr(W_lo),
                                    float(mass), _ptr(b), _ptr(x), nrhs, _ptr(work), nbytes,
                                    ctypes.byref(stats), _stream())
    info = {
        "iterations": stats.iterations, "outer": stats.outer, "applies": stats.applies,
        "converged": bool(stats.converged),
        "true_residual": [stats.true_residual[i] for i in range(min(nrhs, _lib.BRI_MAX_RHS))],
        "status": st,
    }
    if st != 0 and (raise_on_noconv or st != -4):
        raise BriError(st, "bri_solve_cgne")
    return x, info


# ------------------------------------------------------------------ production operator (Sec. 5)
def bri_project_su3(A, out=None):
    """Closest SU(3) matrices for FP64 SoA matrices A [9, n, 2]; out may be A."""
    _need_cuda(A, out)
    if prec_of(A) != F64 or A.dim() != 3 or A.shape[0] != 9 or A.shape[2] != 2:
        raise ValueError("A must be an FP64 tensor [9, n, 2]")
    Y = out if out is not None else torch.empty_like(A)
    _shape(Y, A.shape, "out")
    _check(_lib_handle.bri_project_su3(A.shape[1], _ptr(A), _ptr(Y), _stream()), "bri_project_su3")
    return Y


def bri_ape_smear(dims, U_soa, alpha=0.72, out=None):
    """One APE smearing step of FP64 SoA links."""
    _need_cuda(U_soa, out)
    _shape(U_soa, (4, 9, volume(dims), 2), "links")
    if prec_of(U_soa) != F64:
        raise ValueError("APE smearing takes FP64 links")
    V = out if out is not None else torch.empty_like(U_soa)
    _shape(V, U_soa.shape, "out")
    _check(_lib_handle.bri_ape_smear(_dims(dims), _ptr(U_soa), _ptr(V), float(alpha), _stream()),
           "bri_ape_smear")
    return V


def _rows(form):
    return 6 if form == W_SU3_2ROW else 9


def bri_build_transporters_ex(dims, U_soa, prec=F64, n_offsets=80, form=W_SU3, out=None):
    _need_cuda(U_soa, out)
    if prec_of(U_soa) != F64:
        raise ValueError("transporters are built from FP64 links")
    _shape(U_soa, (4, 9, volume(dims), 2), "links")
    shape = (n_offsets, _rows(form), volume(dims), 2)
    W = out if out is not None else torch.empty(shape, dtype=_TORCH[prec], device=U_soa.device)
    _shape(W, shape, "transporters")
    nbytes = _lib_handle.bri_build_workspace_bytes_ex(_dims(dims), prec, n_offsets, form)
    work = torch.empty(max(nbytes, 16), dtype=torch.uint8, device=U_soa.device) if nbytes else None
    _check(_lib_handle.bri_build_transporters_ex(_dims(dims), _ptr(U_soa), _ptr(W), prec, n_offsets, form,
                                                 _ptr(work), nbytes, _stream()),
           "bri_build_transporters_ex")
    return W


def bri_build_clover(dims, U_soa, csw=1.0, prec=F64):
    """Clover term [2, 18, V, 2] in prec from FP64 SoA links."""
    _need_cuda(U_soa)
    _shape(U_soa, (4, 9, volume(dims), 2), "links")
    if prec_of(U_soa) != F64:
        raise ValueError("the clover term is built from FP64 links")
    C = torch.empty((2, 18, volume(dims), 2), dtype=_TORCH[prec], device=U_soa.device)
    _check(_lib_handle.bri_build_clover(_dims(dims), _ptr(U_soa), float(csw), _ptr(C), prec, _stream()),
           "bri_build_clover")
    return C


# Coefficient tables of the generic ultralocal class (Sec. 8, Tab. rholambda):
# (lambda_0, lambda_1, lambda_2, lambda_3, lambda_4, rho_1, rho_2, rho_3, rho_4).
TABLE_WILSON = (4.0, -0.5, 0.0, 0.0, 0.0, 0.5, 0.0, 0.0, 0.0)
TABLE_HYPERCUBE = (1.852720547, -0.060757866, -0.030036032, -0.015967620, -0.008426812,
                   0.136846794, 0.032077284, 0.011058131, 0.004748991)
TABLE_BRILLOUIN = (240 / 128, -8 / 128, -4 / 128, -2 / 128, -1 / 128, 64 / 432, 16 / 432, 4 / 432, 1 / 432)


class Operator:
    """Transporters (and form) plus an optional clover term and an optional
    coefficient table of the generic class (nine numbers, lambda_0..4 then
    rho_1..4; None is the Brillouin operator); keeps the tensors alive."""

    def __init__(self, W, form=W_AVERAGE, clover=None, coef=None):
        self.W, self.form, self.clover = W, form, clover
        if coef is not None:
            coef = tuple(float(c) for c in coef)
            if len(coef) != 9:
                raise ValueError("a coefficient table has nine entries (lambda_0..4, rho_1..4)")
            self._coef_c = (ctypes.c_double * 9)(*coef)
        self.coef = coef

    def struct(self, dims):
        _need_cuda(self.W, self.clover)
        V = volume(dims)
        _shape(self.W, (self.W.shape[0], _rows(self.form), V, 2), "transporters")
        if self.clover is not None:
            _shape(self.clover, (2, 18, V, 2), "clover")
        o = _lib.bri_operator()
        o.W = self.W.data_ptr()
        o.w_prec = prec_of(self.W)
        o.n_offsets = self.W.shape[0]
        o.w_form = self.form
        o.clover = self.clover.data_ptr() if self.clover is not None else None
        o.coef = ctypes.addressof(self._coef_c) if self.coef is not None else None
        return o


def bri_apply_op(dims, op, psi, mass, dagger=False, out=None):
    """out = D psi (or D^dag psi) for an Operator."""
    _need_cuda(psi, out)
    _shape(psi, (psi.shape[0], 12, volume(dims), 2), "spinor")
    if op.clover is not None and op.clover.dtype != psi.dtype:
        raise ValueError("the clover term must be stored in the spinor precision")
    if out is None:
        out = torch.empty_like(psi)
    elif out.shape != psi.shape or out.dtype != psi.dtype:
        raise ValueError("out must match the input spinor's shape and dtype")
    o = op.struct(dims)
    _check(_lib_handle.bri_apply_op(_dims(dims), ctypes.byref(o), prec_of(psi), float(mass), _ptr(psi),
                                    _ptr(out), psi.shape[0], int(bool(dagger)), _stream()),
           "bri_apply_op")
    return out


def bri_solve_cgne_op(dims, op_hi, b, mass, params, op_lo=None, x=None, raise_on_noconv=True):
    """bri_solve_cgne for Operators (op_hi FP64; op_lo in the inner precision,
    clover FP32).  Returns (x, stats dict)."""
    _need_cuda(b, x)
    V = volume(dims)
    _shape(b, (b.shape[0], 12, V, 2), "b")
    if x is not None:
        _shape(x, b.shape, "x")
    if prec_of(b) != F64 or prec_of(op_hi.W) != F64:
        raise ValueError("b and the outer operator must be FP64")
    if op_hi.clover is not None and op_hi.clover.dtype != torch.float64:
        raise ValueError("the outer clover term must be FP64")
    if params.inner_prec != F64:
        if op_lo is None or prec_of(op_lo.W) != params.inner_prec:
            raise ValueError("op_lo must be given in the inner precision")
        if op_lo.clover is not None and op_lo.clover.dtype != torch.float32:
            raise ValueError("the inner clover term must be FP32")
    nrhs = b.shape[0]
    if x is None:
        x = torch.zeros_like(b)
    nbytes = _lib_handle.bri_solve_workspace_bytes(_dims(dims), ctypes.byref(params), nrhs)
    work = torch.empty(max(nbytes, 16), dtype=torch.uint8, device=b.device)
    stats = _lib.bri_solve_stats()
    hi = op_hi.struct(dims)
    lo = op_lo.struct(dims) if op_lo is not None else None
    st = _lib_handle.bri_solve_cgne_op(_dims(dims), ctypes.byref(params), ctypes.byref(hi),
                                       ctypes.byref(lo) if lo is not None else None, float(mass), _ptr(b),
                                       _ptr(x), nrhs, _ptr(work), nbytes, ctypes.byref(stats), _stream())
    info = {
        "iterations": stats.iterations, "outer": stats.outer, "applies": stats.applies,
        "converged": bool(stats.converged),
        "true_residual": [stats.true_residual[i] for i in range(min(nrhs, _lib.BRI_MAX_RHS))],
        "status": st,
    }
    if st != 0 and (raise_on_noconv or st != -4):
        raise BriError(st, "bri_solve_cgne_op")
    return x, info


# ------------------------------------------------------------------ overlap operator (Sec. 7)
def bri_lanczos(dims, op, mass, k, v0, keep_basis=False):
    """k Lanczos steps on D^dag D (op at `mass`) from the FP64 field v0 [1,12,V,2].
    Returns (alpha, beta, basis or None) with numpy alpha, beta truncated to
    the steps performed."""
    import numpy as np
    _need_cuda(v0)
    _shape(v0, (1, 12, volume(dims), 2), "v0")
    if prec_of(v0) != F64:
        raise ValueError("the Lanczos process works on FP64 fields")
    alpha = np.zeros(k)
    beta = np.zeros(k)
    basis = torch.empty((k, 12, volume(dims), 2), dtype=torch.float64, device=v0.device) if keep_basis else None
    nbytes = _lib_handle.bri_lanczos_workspace_bytes(_dims(dims), int(k))
    work = torch.empty(max(nbytes, 16), dtype=torch.uint8, device=v0.device)
    done = ctypes.c_int32(0)
    o = op.struct(dims)
    _check(_lib_handle.bri_lanczos(_dims(dims), ctypes.byref(o), float(mass), int(k), _ptr(v0),
                                   alpha.ctypes.data_as(ctypes.c_void_p), beta.ctypes.data_as(ctypes.c_void_p),
                                   _ptr(basis), ctypes.byref(done), _ptr(work), nbytes, _stream()), "bri_lanczos")
    n = done.value
    return alpha[:n], beta[:n], (basis[:n] if basis is not None else None)


def bri_ritz_values(alpha, beta, filter=True):
    """Eigenvalues of the Lanczos tridiagonal (ascending), optionally with
    spurious copies removed."""
    import numpy as np
    a = np.ascontiguousarray(alpha, dtype=np.float64)
    b = np.ascontiguousarray(beta, dtype=np.float64)
    out = np.zeros(len(a))
    n = ctypes.c_int32(0)
    _check(_lib_handle.bri_ritz_values(len(a), a.ctypes.data_as(ctypes.c_void_p), b.ctypes.data_as(ctypes.c_void_p),
                                       int(bool(filter)), out.ctypes.data_as(ctypes.c_void_p), ctypes.byref(n)),
           "bri_ritz_values")
    return out[:n.value]


def bri_overlap_lowmodes(dims, op, mass, k, v0, n_low):
    """The n_low eigenmodes of gamma5 D (op at `mass`) of smallest |eigenvalue|.
    Returns (vecs [n_low,12,V,2] FP64, evals numpy, residuals numpy)."""
    import numpy as np
    _need_cuda(v0)
    V = volume(dims)
    _shape(v0, (1, 12, V, 2), "v0")
    basis = torch.empty((k, 12, V, 2), dtype=torch.float64, device=v0.device)
    vecs = torch.empty((n_low, 12, V, 2), dtype=torch.float64, device=v0.device)
    ev = np.zeros(n_low)
    rs = np.zeros(n_low)
    nbytes = _lib_handle.bri_lowmodes_workspace_bytes(_dims(dims), int(k), int(n_low))
    work = torch.empty(max(nbytes, 16), dtype=torch.uint8, device=v0.device)
    o = op.struct(dims)
    _check(_lib_handle.bri_overlap_lowmodes(_dims(dims), ctypes.byref(o), float(mass), int(k), _ptr(v0), int(n_low),
                                            _ptr(basis), _ptr(vecs), ev.ctypes.data_as(ctypes.c_void_p),
                                            rs.ctypes.data_as(ctypes.c_void_p), _ptr(work), nbytes, _stream()),
           "bri_overlap_lowmodes")
    del basis
    return vecs, ev, rs


def bri_sign_approx_error(lo, hi, degree):
    """max over [lo, hi] of |1 - sqrt(x) p(x)| for the degree-`degree` interpolant."""
    e = ctypes.c_double(0.0)
    _check(_lib_handle.bri_sign_approx_error(float(lo), float(hi), int(degree), ctypes.byref(e)),
           "bri_sign_approx_error")
    return e.value


def sign_degree(lo, hi, target, max_degree=100000):
    """Smallest degree (doubling from 16, then bisection) whose error bound is below target."""
    lo_d, d = 0, 16
    while bri_sign_approx_error(lo, hi, d) >= target:
        lo_d, d = d, 2 * d
        if d > max_degree:
            raise ValueError("the interval needs a degree above max_degree")
    while d - lo_d > 1:
        m = (lo_d + d) // 2
        if bri_sign_approx_error(lo, hi, m) < target:
            d = m
        else:
            lo_d = m
    return d


def _lowmodes(dims, low_vecs, low_evals):
    import numpy as np
    if low_vecs is None or len(low_evals) == 0:
        return 0, None, None
    _need_cuda(low_vecs)
    _shape(low_vecs, (len(low_evals), 12, volume(dims), 2), "low_vecs")
    ev = np.ascontiguousarray(low_evals, dtype=np.float64)
    return len(ev), low_vecs, ev


def bri_sign_h(dims, op, mass, psi, lo, hi, degree, low_vecs=None, low_evals=(), out=None, with_error=True):
    """sign(gamma5 D) psi for FP64 fields; returns (out, approx_err) (approx_err
    None when with_error is False, which skips its host-side evaluation)."""
    _need_cuda(psi, out)
    _shape(psi, (psi.shape[0], 12, volume(dims), 2), "psi")
    if prec_of(psi) != F64:
        raise ValueError("sign(H) works on FP64 fields")
    n_low, lv, ev = _lowmodes(dims, low_vecs, low_evals)
    out = out if out is not None else torch.empty_like(psi)
    nbytes = _lib_handle.bri_sign_workspace_bytes(_dims(dims), psi.shape[0])
    work = torch.empty(max(nbytes, 16), dtype=torch.uint8, device=psi.device)
    err = ctypes.c_double(0.0)
    o = op.struct(dims)
    _check(_lib_handle.bri_sign_h(_dims(dims), ctypes.byref(o), float(mass), float(lo), float(hi), int(degree),
                                  n_low, _ptr(lv), ev.ctypes.data_as(ctypes.c_void_p) if ev is not None else None,
                                  _ptr(psi), _ptr(out), psi.shape[0], ctypes.byref(err) if with_error else None,
                                  _ptr(work), nbytes, _stream()), "bri_sign_h")
    return out, (err.value if with_error else None)


def bri_overlap_apply(dims, op, psi, rho, m, lo, hi, degree, low_vecs=None, low_evals=(), out=None):
    """D_ov,m psi (Eqs. def_over, def_mass) for FP64 fields; returns (out, approx_err)."""
    _need_cuda(psi, out)
    _shape(psi, (psi.shape[0], 12, volume(dims), 2), "psi")
    if prec_of(psi) != F64:
        raise ValueError("the overlap operator works on FP64 fields")
    n_low, lv, ev = _lowmodes(dims, low_vecs, low_evals)
    out = out if out is not None else torch.empty_like(psi)
    nbytes = _lib_handle.bri_sign_workspace_bytes(_dims(dims), psi.shape[0])
    work = torch.empty(max(nbytes, 16), dtype=torch.uint8, device=psi.device)
    err = ctypes.c_double(0.0)
    o = op.struct(dims)
    _check(_lib_handle.bri_overlap_apply(_dims(dims), ctypes.byref(o), float(rho), float(m), float(lo), float(hi),
                                         int(degree), n_low, _ptr(lv),
                                         ev.ctypes.data_as(ctypes.c_void_p) if ev is not None else None,
                                         _ptr(psi), _ptr(out), psi.shape[0], ctypes.byref(err), _ptr(work),
                                         nbytes, _stream()), "bri_overlap_apply")
    return out, err.value


# ------------------------------------------------------------------ gradient
def bri_grad_links(dims, U_soa, chi, psi, scale=1.0, W40=None, coef=None):
    """scale * dS/dU (FP64 SoA links) for S = Re sum_rhs <chi, D psi>.  W40:
    the FP64 40-offset transporters of U if already built (else rebuilt).
    coef: None for the Brillouin operator, or a generic-class table (nine
    numbers, as for Operator)."""
    _need_cuda(U_soa, chi, psi)
    V = volume(dims)
    _shape(U_soa, (4, 9, V, 2), "links")
    _shape(chi, (chi.shape[0], 12, V, 2), "chi")
    _shape(psi, chi.shape, "psi")
    if prec_of(U_soa) != F64 or prec_of(chi) != F64 or prec_of(psi) != F64:
        raise ValueError("the link gradient is FP64")
    g = torch.empty_like(U_soa)
    cf = None
    if coef is not None:
        coef = tuple(float(c) for c in coef)
        if len(coef) != 9:
            raise ValueError("a coefficient table has nine entries (lambda_0..4, rho_1..4)")
        cf = (ctypes.c_double * 9)(*coef)
    if W40 is not None:
        _need_cuda(W40)
        _shape(W40, (40, 9, V, 2), "W40")
        if prec_of(W40) != F64:
            raise ValueError("W40 must be the FP64 40-offset store")
        nbytes = _lib_handle.bri_grad_workspace_bytes_w(_dims(dims))
        work = torch.empty(max(nbytes, 16), dtype=torch.uint8, device=U_soa.device)
        _check(_lib_handle.bri_grad_links_w(_dims(dims), _ptr(U_soa), _ptr(W40), _ptr(chi), _ptr(psi),
                                            chi.shape[0], float(scale), cf, _ptr(g), _ptr(work), nbytes,
                                            _stream()),
               "bri_grad_links_w")
        return g
    nbytes = _lib_handle.bri_grad_workspace_bytes(_dims(dims))
    work = torch.empty(max(nbytes, 16), dtype=torch.uint8, device=U_soa.device)
    _check(_lib_handle.bri_grad_links(_dims(dims), _ptr(U_soa), _ptr(chi), _ptr(psi), chi.shape[0],
                                      float(scale), cf, _ptr(g), _ptr(work), nbytes, _stream()),
           "bri_grad_links")
    return g
