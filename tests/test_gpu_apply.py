"""GPU parity: transporter construction and operator application through the
C ABI against the FP64 CPU oracle, on seeded synthetic inputs.

Tolerances (relative, in the 2-norm over the whole output, and element by
element against the largest reference element):
  FP64 storage/arithmetic                         1e-12
  FP32 storage, FP32 accumulation                 1e-5
  FP16 transporters (FP32 or FP16 spinors),
  FP32 accumulation                               5e-3
The FP32 bound is ~100x the expected error (u_32 = 6e-8 times the growth of a
sum of 81 terms); FP16 storage rounds every W element with u_16 = 4.9e-4.
"""
import numpy as np
import pytest

import synth
from oracle import dirac, transporters as otr
from tests.helpers import (dev, host, log, plane_offsets, rel, soa_to_canon,
                           transporter_plane_to_canon)

pytestmark = pytest.mark.gpu

TOL = {("f64", "f64"): 1e-12, ("f32", "f32"): 1e-5, ("f16", "f32"): 5e-3, ("f16", "f16"): 5e-3}
PREC = {"f64": 0, "f32": 1, "f16": 2}

# lattices: the 4^4 case, ragged volumes (not multiples of the 256-thread
# block), extent-2 directions (x+1 == x-1), a multi-block case, and two
# lattices with Lx a multiple of 32 and Ly of 16, where the FP32 and FP64
# 80-offset apply with one right-hand side takes the 32x16 tile that the
# benchmark times at 32^3 x 64 (one tile per (z, t); the second with z and t
# of extent 2, so the tile's z and t neighbours wrap onto one slice).  With
# Lx a multiple of 16 the transporter build and the recompute apply order
# their 16-site x strips in groups of Lx/16 x gy x gz strips (gy, gz = 4, 2 or
# 1 by divisibility): (16, 6, 2, 2) takes 2 x 2, (32, 16, 3, 4) 4 x 1,
# (32, 16, 2, 2) 4 x 2 and (16, 3, 3, 2) 1 x 1.
LATTICES = [(4, 4, 4, 4), (5, 3, 2, 6), (2, 2, 2, 2), (6, 4, 4, 8), (16, 6, 2, 2), (32, 16, 3, 4),
            (32, 16, 2, 2), (16, 3, 3, 2)]


@pytest.fixture(scope="module")
def bri():
    import paper_1012_3615_amd as m
    return m


_cache = {}


def setup_case(dims, eps=0.3, seed=1001, nrhs=1, mass=0.1):
    key = (dims, eps, seed, nrhs)
    if key not in _cache:
        u = synth.gauge_links(dims, eps, seed)
        psi = synth.gaussian_spinor(dims, seed + 1, nrhs=nrhs)
        ref = np.stack([dirac.apply(u, psi[r], mass) for r in range(nrhs)])
        refd = np.stack([dirac.apply_dag(u, psi[r], mass) for r in range(nrhs)])
        _cache[key] = (u, psi, ref, refd)
    return _cache[key]


def check(out, ref, tol, what):
    r = rel(out, ref)
    emax = float(np.abs(out - ref).max() / np.abs(ref).max())
    assert r <= tol and emax <= 10 * tol, f"{what}: rel {r:.3e} max-elem {emax:.3e} > {tol}"
    return r


@pytest.mark.parametrize("dims", LATTICES)
def test_transporters_match_oracle(bri, dims):
    log(f"build transporters FP64 dims={dims}")
    u = synth.gauge_links(dims, 0.4, 7)
    U = bri.bri_pack_links(dims, dev(u), bri.F64)
    W80 = bri.bri_build_transporters(dims, U, bri.F64, 80)
    W40 = bri.bri_build_transporters(dims, U, bri.F64, 40)
    import torch
    torch.cuda.synchronize()
    for j, n in enumerate(plane_offsets(80)):
        ref = otr.transporter(u, n)
        got = transporter_plane_to_canon(dims, W80[j])
        assert np.abs(got - ref).max() < 1e-14, (n, np.abs(got - ref).max())
    for c, n in enumerate(plane_offsets(40)):
        j = plane_offsets(80).index(n)
        assert torch.equal(W40[c], W80[j])


@pytest.mark.parametrize("dims", LATTICES)
@pytest.mark.parametrize("wp,sp", [("f64", "f64"), ("f32", "f32"), ("f16", "f32"), ("f16", "f16")])
@pytest.mark.parametrize("noff", [80, 40])
def test_apply_stored_matches_oracle(bri, dims, wp, sp, noff):
    u, psi, ref, refd = setup_case(dims)
    log(f"apply stored dims={dims} W={wp} psi={sp} noff={noff}")
    U = bri.bri_pack_links(dims, dev(u), bri.F64)
    W = bri.bri_build_transporters(dims, U, PREC[wp], noff)
    x = bri.bri_pack_spinor(dims, dev(psi), PREC[sp])
    if dims[0] % 32 == 0 and dims[1] % 16 == 0 and noff == 80 and wp == sp and wp != "f16":
        assert bri.bri_get_apply_config(dims, PREC[wp], PREC[sp], noff, 1) == (13, 1)
    out = bri.bri_apply(dims, W, x, 0.1)
    outd = bri.bri_apply_dag(dims, W, x, 0.1)
    tol = TOL[(wp, sp)]
    check(soa_to_canon(dims, out), ref, tol, "D")
    check(soa_to_canon(dims, outd), refd, tol, "D^dag")


@pytest.mark.parametrize("dims", LATTICES)
@pytest.mark.parametrize("p", ["f64", "f32"])
def test_apply_recompute_matches_oracle(bri, dims, p):
    u, psi, ref, refd = setup_case(dims)
    log(f"apply recompute dims={dims} prec={p}")
    U = bri.bri_pack_links(dims, dev(u), PREC[p])
    x = bri.bri_pack_spinor(dims, dev(psi), PREC[p])
    out = bri.bri_apply(dims, U, x, 0.1, variant=bri.RECOMPUTE)
    outd = bri.bri_apply_dag(dims, U, x, 0.1, variant=bri.RECOMPUTE)
    tol = TOL[(p, p)]
    check(soa_to_canon(dims, out), ref, tol, "D")
    check(soa_to_canon(dims, outd), refd, tol, "D^dag")


def test_unpack_roundtrip(bri):
    dims = (5, 3, 2, 6)
    psi = synth.gaussian_spinor(dims, 5, nrhs=3)
    log("pack/unpack roundtrip")
    x = bri.bri_pack_spinor(dims, dev(psi), bri.F64)
    assert np.array_equal(soa_to_canon(dims, x), psi)
    back = host(bri.bri_unpack_spinor(dims, x))
    assert np.array_equal(back, psi)


@pytest.mark.parametrize("wp,sp", [("f64", "f64"), ("f32", "f32"), ("f16", "f32")])
@pytest.mark.parametrize("rblk", [1, 2, 3, 4, 6, 12])
def test_multi_rhs_point_sources(bri, wp, sp, rblk):
    """The 12 spin-colour point sources in one fused launch, for every
    rhs-per-thread blocking; each column must match the oracle."""
    dims = (4, 4, 2, 6)
    u = synth.gauge_links(dims, 0.3, 4001)
    src = synth.point_sources(dims, site=(1, 2, 1, 3))
    key = ("ps", dims)
    if key not in _cache:
        _cache[key] = np.stack([dirac.apply(u, src[r], 0.1) for r in range(12)])
    ref = _cache[key]
    log(f"multi-rhs W={wp} psi={sp} rblk={rblk}")
    U = bri.bri_pack_links(dims, dev(u), bri.F64)
    W = bri.bri_build_transporters(dims, U, PREC[wp], 80)
    x = bri.bri_pack_spinor(dims, dev(src), PREC[sp])
    try:
        bri.bri_set_apply_config(dims, PREC[wp], PREC[sp], 80, 12, 1, rblk)
        out = bri.bri_apply(dims, W, x, 0.1)
    finally:
        bri.bri_clear_apply_configs()
    got = soa_to_canon(dims, out)
    for r in range(12):
        check(got[r], ref[r], TOL[(wp, sp)], f"rhs {r}")
    # blocking does not change the arithmetic of a column
    one = soa_to_canon(dims, bri.bri_apply(dims, W, x[5:6].contiguous(), 0.1))
    assert np.array_equal(one[0], got[5])


@pytest.mark.parametrize("wp,sp", [("f64", "f64"), ("f32", "f32"), ("f16", "f32")])
@pytest.mark.parametrize("kind", ["point", "gaussian"])
def test_multi_rhs_default_launch_lx32(bri, wp, sp, kind):
    """Twelve right-hand sides in one fused launch with the built-in selection
    at Lx = 32 (the 32x8 tile with prefetch and unrolled offsets, two
    right-hand sides per thread: the configuration the autotuner picks for
    the 12-source apply at 32^3 x 64), D and D^dag, every column element by
    element against the oracle.  The point sources sit on a tile corner
    (x = 31, y = 7), so their 81-point images wrap across tile and lattice
    edges; the Gaussian fields load every tile."""
    dims = (32, 8, 2, 3)
    u = synth.gauge_links(dims, 0.3, 4001)
    if kind == "point":
        src = synth.point_sources(dims, site=(31, 7, 1, 2))
    else:
        src = synth.gaussian_spinor(dims, 4012, nrhs=12)
    key = ("lx32", kind, dims)
    if key not in _cache:
        _cache[key] = (np.stack([dirac.apply(u, src[r], 0.1) for r in range(12)]),
                       np.stack([dirac.apply_dag(u, src[r], 0.1) for r in range(12)]))
    ref, refd = _cache[key]
    log(f"multi-rhs default launch Lx=32 W={wp} psi={sp} {kind}")
    bri.bri_clear_apply_configs()
    assert bri.bri_get_apply_config(dims, PREC[wp], PREC[sp], 80, 12) == (8, 2)
    U = bri.bri_pack_links(dims, dev(u), bri.F64)
    W = bri.bri_build_transporters(dims, U, PREC[wp], 80)
    x = bri.bri_pack_spinor(dims, dev(src), PREC[sp])
    got = soa_to_canon(dims, bri.bri_apply(dims, W, x, 0.1))
    gotd = soa_to_canon(dims, bri.bri_apply_dag(dims, W, x, 0.1))
    for r in range(12):
        check(got[r], ref[r], TOL[(wp, sp)], f"D rhs {r}")
        check(gotd[r], refd[r], TOL[(wp, sp)], f"D^dag rhs {r}")


def test_multi_rhs_ragged_count(bri):
    """nrhs = 7 with 4 rhs per thread: the last group is partial."""
    dims = (4, 4, 4, 4)
    u, _, _, _ = setup_case(dims)
    psi = synth.gaussian_spinor(dims, 77, nrhs=7)
    log("multi-rhs nrhs=7 rblk=4")
    U = bri.bri_pack_links(dims, dev(u), bri.F64)
    W = bri.bri_build_transporters(dims, U, bri.F32, 80)
    x = bri.bri_pack_spinor(dims, dev(psi), bri.F32)
    try:
        bri.bri_set_apply_config(dims, bri.F32, bri.F32, 80, 7, 1, 4)
        assert bri.bri_get_apply_config(dims, bri.F32, bri.F32, 80, 7) == (10, 4)
        out = soa_to_canon(dims, bri.bri_apply(dims, W, x, 0.1))
    finally:
        bri.bri_clear_apply_configs()
    for r in range(7):
        check(out[r], dirac.apply(u, psi[r], 0.1), 1e-5, f"rhs {r}")


def test_gamma5_hermiticity_and_gauge_covariance_on_gpu(bri):
    """Properties of the GPU output itself (FP64): <chi, D psi> = <D^dag chi, psi>
    and D[U^g](g psi) = g D[U] psi."""
    dims = (6, 4, 4, 6)
    u = synth.gauge_links(dims, 0.4, 55)
    psi = synth.gaussian_spinor(dims, 56)
    chi = synth.gaussian_spinor(dims, 57)
    g = synth.random_su3_field(dims, 58)
    log("gpu properties gamma5/gauge")
    U = bri.bri_pack_links(dims, dev(u), bri.F64)
    W = bri.bri_build_transporters(dims, U, bri.F64, 40)
    xp = bri.bri_pack_spinor(dims, dev(psi), bri.F64)
    xc = bri.bri_pack_spinor(dims, dev(chi), bri.F64)
    dpsi = soa_to_canon(dims, bri.bri_apply(dims, W, xp, 0.2))[0]
    ddchi = soa_to_canon(dims, bri.bri_apply_dag(dims, W, xc, 0.2))[0]
    a, b = np.vdot(chi, dpsi), np.vdot(ddchi, psi)
    assert abs(a - b) / abs(a) < 1e-13
    ug = synth.gauge_transform_links(u, g)
    Ug = bri.bri_pack_links(dims, dev(ug), bri.F64)
    Wg = bri.bri_build_transporters(dims, Ug, bri.F64, 80)
    xg = bri.bri_pack_spinor(dims, dev(synth.gauge_transform_spinor(psi, g)), bri.F64)
    lhs = soa_to_canon(dims, bri.bri_apply(dims, Wg, xg, 0.2))[0]
    assert rel(lhs, synth.gauge_transform_spinor(dpsi, g)) < 1e-13


def test_error_paths(bri):
    import torch
    dims = (4, 4, 4, 4)
    u, psi, _, _ = setup_case(dims)
    log("error paths")
    U = bri.bri_pack_links(dims, dev(u), bri.F64)
    W = bri.bri_build_transporters(dims, U, bri.F32, 80)
    x = bri.bri_pack_spinor(dims, dev(psi), bri.F32)
    with pytest.raises(bri.BriError) as e:
        bri.bri_apply(dims, W, x, 0.1, out=x)
    assert e.value.status == -1
    with pytest.raises(bri.BriError):
        bri.bri_apply(dims, W[:39].contiguous(), x, 0.1)   # 39 offsets
    x64 = bri.bri_pack_spinor(dims, dev(psi), bri.F64)
    with pytest.raises(bri.BriError) as e:
        bri.bri_apply(dims, W, x64, 0.1)                      # F32 W with F64 spinors
    assert e.value.status == -2
    with pytest.raises(ValueError):
        bri.bri_apply((4, 4, 4, 2), W, x, 0.1)                # buffers too small for dims
    # the C ABI itself rejects an extent < 2 before touching memory
    import ctypes
    from paper_1012_3615_amd import _lib
    d = _lib.bri_dims()
    d.L[0], d.L[1], d.L[2], d.L[3] = 4, 4, 16, 1
    y = torch.empty_like(x)
    st = bri.api.lib().bri_apply(d, 0, ctypes.c_void_p(W.data_ptr()), 1, 80, 1, 0.1,
                                 ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()), 1,
                                 None)
    assert st == -1
