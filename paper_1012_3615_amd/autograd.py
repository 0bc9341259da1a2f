"""torch.autograd Functions over the HIP library (FP64).

PyTorch's complex gradients are g = dL/dRe z + i dL/dIm z for a real loss L,
and the incoming grad_output of out = D[U] psi plays the role of chi in
S = Re <chi, D psi>.  Hence

    d/dpsi :  D^dag grad_output            (bri_apply_dag)
    d/dU   :  link gradient of Re <grad_output, D psi>   (bri_grad_links)

The transporters are rebuilt from U in the backward pass (once, as the FP64
40-offset store shared by the psi gradient and the link gradient); only U and
psi are saved.  All tensors are canonical complex128 device tensors:
U [4, Lt, Lz, Ly, Lx, 3, 3], fields [nrhs, Lt, Lz, Ly, Lx, 4, 3].
"""
from __future__ import annotations

import torch

from . import api


def _dims_of(U):
    return (U.shape[4], U.shape[3], U.shape[2], U.shape[1])


class BriApply(torch.autograd.Function):
    """out = D[U] psi (Eq. def_pref, c_SW = 0); with `coef`, any member of the
    generic class of Sec. 8 (nine numbers, lambda_0..4 then rho_1..4)."""

    @staticmethod
    def forward(ctx, U, psi, mass, n_offsets=80, coef=None):
        dims = _dims_of(U)
        Us = api.bri_pack_links(dims, U.contiguous(), api.F64)
        W = api.bri_build_transporters(dims, Us, api.F64, n_offsets)
        x = api.bri_pack_spinor(dims, psi.contiguous(), api.F64)
        y = api.bri_apply(dims, W, x, mass) if coef is None else api.bri_apply_op(dims, api.Operator(W, coef=coef), x, mass)
        out = api.bri_unpack_spinor(dims, y)
        ctx.save_for_backward(U, psi)
        ctx.mass, ctx.noff, ctx.coef = mass, n_offsets, coef
        return out.reshape(psi.shape)

    @staticmethod
    def backward(ctx, gout):
        U, psi = ctx.saved_tensors
        dims = _dims_of(U)
        Us = api.bri_pack_links(dims, U.contiguous(), api.F64)
        chi = api.bri_pack_spinor(dims, gout.contiguous(), api.F64)
        gU = gpsi = None
        W40 = api.bri_build_transporters(dims, Us, api.F64, 40)
        if ctx.needs_input_grad[1]:
            if ctx.coef is None:
                y = api.bri_apply_dag(dims, W40, chi, ctx.mass)
            else:
                y = api.bri_apply_op(dims, api.Operator(W40, coef=ctx.coef), chi, ctx.mass, dagger=True)
            gpsi = api.bri_unpack_spinor(dims, y).reshape(psi.shape)
        if ctx.needs_input_grad[0]:
            x = api.bri_pack_spinor(dims, psi.contiguous(), api.F64)
            gU = api.bri_unpack_links(dims, api.bri_grad_links(dims, Us, chi, x, W40=W40, coef=ctx.coef))
        return gU, gpsi, None, None, None


def _solve_normal(dims, W, b_soa, mass, tol, n_offsets):
    """(D^dag D)^{-1} b: first D^dag y = b, then D x = y (FP64 CGNE)."""
    p = api.solve_params(tol=tol, inner_prec=api.F64, n_offsets=n_offsets, dagger=True)
    y, _ = api.bri_solve_cgne(dims, W, b_soa, mass, p)
    p = api.solve_params(tol=tol, inner_prec=api.F64, n_offsets=n_offsets)
    x, _ = api.bri_solve_cgne(dims, W, y, mass, p)
    return x


class BriNormalSolve(torch.autograd.Function):
    """X = (D^dag D)^{-1} phi, differentiable in U and phi.

    With M = D^dag D and Y = M^{-1} grad_X: grad_phi = Y and
    grad_U = -[link gradient of Re<D X, D Y> in the second factor
               + link gradient of Re<D Y, D X> in the second factor],
    i.e. bri_grad_links with (chi, psi) = ([D X, D Y], [Y, X])."""

    @staticmethod
    def forward(ctx, U, phi, mass, tol=1e-13, n_offsets=80):
        dims = _dims_of(U)
        Us = api.bri_pack_links(dims, U.contiguous(), api.F64)
        W = api.bri_build_transporters(dims, Us, api.F64, n_offsets)
        b = api.bri_pack_spinor(dims, phi.contiguous(), api.F64)
        X = _solve_normal(dims, W, b, mass, tol, n_offsets)
        ctx.save_for_backward(U, api.bri_unpack_spinor(dims, X))
        ctx.mass, ctx.tol, ctx.noff = mass, tol, n_offsets
        return api.bri_unpack_spinor(dims, X).reshape(phi.shape)

    @staticmethod
    def backward(ctx, gX):
        U, Xc = ctx.saved_tensors
        dims = _dims_of(U)
        Us = api.bri_pack_links(dims, U.contiguous(), api.F64)
        W = api.bri_build_transporters(dims, Us, api.F64, ctx.noff)
        g = api.bri_pack_spinor(dims, gX.contiguous(), api.F64)
        Y = _solve_normal(dims, W, g, ctx.mass, ctx.tol, ctx.noff)
        gphi = api.bri_unpack_spinor(dims, Y).reshape(gX.shape) if ctx.needs_input_grad[1] else None
        gU = None
        if ctx.needs_input_grad[0]:
            X = api.bri_pack_spinor(dims, Xc.contiguous(), api.F64)
            DX = api.bri_apply(dims, W, X, ctx.mass)
            DY = api.bri_apply(dims, W, Y, ctx.mass)
            chi = torch.cat([DX, DY], dim=0).contiguous()
            psi = torch.cat([Y, X], dim=0).contiguous()
            gU = api.bri_unpack_links(dims, api.bri_grad_links(dims, Us, chi, psi, scale=-1.0))
        return gU, gphi, None, None, None


def apply(U, psi, mass, n_offsets=80, coef=None):
    return BriApply.apply(U, psi, mass, n_offsets, coef)


def normal_solve(U, phi, mass, tol=1e-13, n_offsets=80):
    return BriNormalSolve.apply(U, phi, mass, tol, n_offsets)
