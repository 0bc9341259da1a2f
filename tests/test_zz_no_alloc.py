"""The allocation-free solver entry point (bri_solve_cgne_noalloc), called
through the C ABI, against the solver with a caller workspace
(bri_solve_cgne) on the same inputs: two calls in a row on one device, the
second with a smaller lattice and fewer right-hand sides (the shared static
workspace keeps the first call's contents), and the rejection of a solve
whose workspace exceeds the static array.  Both entry points run the same
kernels on the same workspace layout, so the solutions and the iteration
counts agree bit for bit."""
import ctypes

import numpy as np
import pytest

import synth
from tests.helpers import dev, log

pytestmark = pytest.mark.gpu


def _c_noalloc(bri, dims, params, W_hi, W_lo, mass, b, x):
    import torch
    from paper_1012_3615_amd import _lib
    stats = _lib.bri_solve_stats()
    ptr = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)
    st = bri.api.lib().bri_solve_cgne_noalloc(
        bri.api._dims(dims), ctypes.byref(params), ptr(W_hi), ptr(W_lo), float(mass), ptr(b), ptr(x),
        b.shape[0], ctypes.byref(stats), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st, stats


@pytest.mark.parametrize("first,second", [
    # (dims, nrhs, inner precision) of the two calls
    (((8, 8, 8, 8), 3, 1), ((4, 4, 4, 4), 1, 0)),
    (((8, 4, 4, 8), 2, 0), ((6, 4, 2, 4), 1, 2)),
])
def test_noalloc_solver_matches_workspace_solver(first, second):
    import torch
    import paper_1012_3615_amd as bri
    need = []
    for k, (dims, nrhs, inner) in enumerate((first, second)):
        log(f"noalloc solve call {k}: dims={dims} nrhs={nrhs} inner={inner}")
        u = synth.gauge_links(dims, 0.3, 7001 + k)
        b = bri.bri_pack_spinor(dims, dev(synth.gaussian_spinor(dims, 7011 + k, nrhs=nrhs)), bri.F64)
        U = bri.bri_pack_links(dims, dev(u), bri.F64)
        W_hi = bri.bri_build_transporters(dims, U, bri.F64, 80)
        W_lo = bri.bri_build_transporters(dims, U, inner, 80) if inner != bri.F64 else None
        p = bri.solve_params(tol=1e-10, inner_prec=inner, inner_tol=1e-3 if inner == 1 else 1e-2, check_every=4)
        need.append(bri.api.lib().bri_solve_workspace_bytes(bri.api._dims(dims), ctypes.byref(p), nrhs))
        assert need[-1] <= 128 << 20
        x_ref, info = bri.bri_solve_cgne(dims, W_hi, b, 0.1, p, W_lo=W_lo)
        x = torch.zeros_like(b)
        st, stats = _c_noalloc(bri, dims, p, W_hi, W_lo, 0.1, b, x)
        torch.cuda.synchronize()
        assert st == 0, bri.api.lib().bri_last_error()
        assert torch.equal(x, x_ref)
        assert (stats.iterations, stats.outer, stats.applies, stats.converged) == \
            (info["iterations"], info["outer"], info["applies"], 1)
        for r in range(nrhs):
            assert stats.true_residual[r] == info["true_residual"][r] <= 1e-10
        # the Python binding of the same entry point
        x2, info2 = bri.bri_solve_cgne_noalloc(dims, W_hi, b, 0.1, p, W_lo=W_lo)
        assert torch.equal(x2, x_ref) and info2["iterations"] == info["iterations"]
    assert need[1] < need[0]  # the second call is the smaller one


def test_noalloc_solver_rejects_a_workspace_beyond_its_array():
    """32^3 x 64 with one FP64 right-hand side needs ~2.8 GB of workspace: the
    call fails with BRI_E_WORKSPACE before any device work (its null pointers
    are never touched), and the message states both sizes."""
    import paper_1012_3615_amd as bri
    from paper_1012_3615_amd import _lib
    dims = (32, 32, 32, 64)
    p = bri.solve_params(tol=1e-10)
    stats = _lib.bri_solve_stats()
    log("noalloc solve: oversized request")
    need = bri.api.lib().bri_solve_workspace_bytes(bri.api._dims(dims), ctypes.byref(p), 1)
    assert need > 128 << 20
    st = bri.api.lib().bri_solve_cgne_noalloc(bri.api._dims(dims), ctypes.byref(p), None, None, 0.1, None, None,
                                              1, ctypes.byref(stats), None)
    assert st == -5
    msg = bri.api.lib().bri_last_error().decode()
    assert str(need) in msg and str(128 << 20) in msg, msg
