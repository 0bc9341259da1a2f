"""GPU parity of the generic ultralocal class (Sec. 8, Tab. rholambda): the
stored-transporter apply with a run-time coefficient table (lambda_0..4,
rho_1..4) against the oracle, for the Wilson and hypercube columns and a
random table, with averaged and with back-projected two-row transporters
plus the clover term, and the solver on such an operator.

Tolerances as for the Brillouin operator: FP64 1e-12, FP32 1e-5 (relative
2-norm).  The Brillouin column through the table must reproduce the default
(compile-time coefficient) kernel bit for bit: the two differ only in where
the coefficients are read from."""
import numpy as np
import pytest

import synth
from oracle import production, smearing, ultralocal
from oracle.gamma import gamma5
from tests.helpers import dev, log, soa_to_canon

pytestmark = pytest.mark.gpu

TOL = {0: 1e-12, 1: 1e-5}


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _random_table(seed):
    rng = np.random.default_rng(seed)
    return tuple(float(v) for v in rng.uniform(-1.0, 1.0, 9))


TABLES = {"wilson": ultralocal.WILSON, "hypercube": ultralocal.HYPERCUBE, "random": _random_table(8401)}


@pytest.fixture(scope="module")
def bri():
    import paper_1012_3615_amd as m
    return m


# Lx <= 16: 16x16 / 16x8 tiles; 32, 24, 48: the 32x8, 24x8, 48x4 tiles, each
# with a partial tile in y
@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (6, 5, 3, 4), (32, 3, 2, 2), (24, 3, 2, 2), (48, 2, 2, 2)])
def test_table_apply_matches_oracle(bri, dims):
    mass = 0.1
    u = synth.gauge_links(dims, 0.4, 8402)
    psi = synth.gaussian_spinor(dims, 8403, nrhs=3)
    U = bri.bri_pack_links(dims, dev(u), bri.F64)
    for name, t in TABLES.items():
        want = np.stack([ultralocal.apply(u, psi[r], mass, t) for r in range(3)])
        want_dag = np.stack([ultralocal.apply_dag(u, psi[r], mass, t) for r in range(3)])
        for p, noff in ((0, 80), (1, 80), (0, 40), (1, 40)):
            log(f"generic class {name} {dims} prec={p} noff={noff}")
            op = bri.Operator(bri.bri_build_transporters(dims, U, p, noff), coef=t)
            for nr in (1, 3):
                x = bri.bri_pack_spinor(dims, dev(psi[:nr]), p)
                got = soa_to_canon(dims, bri.bri_apply_op(dims, op, x, mass))
                gdg = soa_to_canon(dims, bri.bri_apply_op(dims, op, x, mass, dagger=True))
                for r in range(nr):
                    assert rel(got[r], want[r]) <= TOL[p], (name, p, noff, nr, r)
                    assert rel(gdg[r], want_dag[r]) <= TOL[p], (name, p, noff, nr, r, "dag")


def test_table_every_kernel_configuration(bri):
    """The table reaches every stored-apply kernel: the gather form (kernel 0,
    several right-hand sides per thread) and each tile shape, against the
    oracle, FP64, 40 and 80 offsets."""
    dims, mass, t = (6, 5, 3, 4), 0.1, TABLES["random"]
    u = synth.gauge_links(dims, 0.4, 8415)
    psi = synth.gaussian_spinor(dims, 8416, nrhs=3)
    want = np.stack([ultralocal.apply(u, psi[r], mass, t) for r in range(3)])
    U = bri.bri_pack_links(dims, dev(u), bri.F64)
    x = bri.bri_pack_spinor(dims, dev(psi), bri.F64)
    try:
        for noff in (80, 40):
            op = bri.Operator(bri.bri_build_transporters(dims, U, bri.F64, noff), coef=t)
            for kernel, rblk in ((0, 3), (0, 1), (2, 2), (3, 1), (5, 3), (8, 2), (9, 3), (10, 2), (11, 1), (12, 2)):
                log(f"generic class kernel {kernel} rblk {rblk} noff {noff}")
                bri.bri_set_apply_config(dims, bri.F64, bri.F64, noff, 3, kernel, rblk)
                got = soa_to_canon(dims, bri.bri_apply_op(dims, op, x, mass))
                for r in range(3):
                    assert rel(got[r], want[r]) <= TOL[0], (kernel, rblk, noff, r)
    finally:
        bri.bri_clear_apply_configs()


@pytest.mark.parametrize("dims", [(8, 4, 4, 4), (32, 4, 2, 2)])
def test_brillouin_table_is_bitwise_the_default(bri, dims):
    u = synth.gauge_links(dims, 0.3, 8404)
    psi = synth.gaussian_spinor(dims, 8405, nrhs=1)
    U = bri.bri_pack_links(dims, dev(u), bri.F64)
    for p in (0, 1):
        log(f"Brillouin table vs default {dims} prec={p}")
        W = bri.bri_build_transporters(dims, U, p, 80)
        x = bri.bri_pack_spinor(dims, dev(psi), p)
        op = bri.Operator(W, coef=bri.TABLE_BRILLOUIN)
        for dag in (False, True):
            ref = (bri.bri_apply_dag if dag else bri.bri_apply)(dims, W, x, 0.1)
            got = bri.bri_apply_op(dims, op, x, 0.1, dagger=dag)
            assert bool((ref == got).all()), (p, dag)


def test_table_with_projected_two_row_and_clover(bri):
    dims, mass = (4, 4, 4, 4), 0.1
    u = synth.gauge_links(dims, 0.4, 8406)
    psi = synth.gaussian_spinor(dims, 8407, nrhs=2)
    us = smearing.ape(u, 0.72)
    Us = bri.bri_ape_smear(dims, bri.bri_pack_links(dims, dev(u), bri.F64), 0.72)
    for name in ("wilson", "hypercube"):
        t = TABLES[name]
        want = np.stack([production.apply(us, psi[r], mass, table=t) for r in range(2)])
        want_dag = np.stack([production.apply_dag(us, psi[r], mass, table=t) for r in range(2)])
        for p in (0, 1):
            log(f"generic class {name} two-row + clover prec={p}")
            op = bri.Operator(bri.bri_build_transporters_ex(dims, Us, p, 80, bri.W_SU3_2ROW), bri.W_SU3_2ROW,
                              bri.bri_build_clover(dims, Us, 1.0, p), coef=t)
            x = bri.bri_pack_spinor(dims, dev(psi), p)
            got = soa_to_canon(dims, bri.bri_apply_op(dims, op, x, mass))
            gdg = soa_to_canon(dims, bri.bri_apply_op(dims, op, x, mass, dagger=True))
            for r in range(2):
                assert rel(got[r], want[r]) <= TOL[p], (name, p, r)
                assert rel(gdg[r], want_dag[r]) <= TOL[p], (name, p, r, "dag")


@pytest.mark.parametrize("inner", [0, 1])
def test_table_solve(bri, inner):
    """CGNE to 1e-10 on the hypercube operator, plain FP64 and with an FP32
    inner solve; the true residual is recomputed with the oracle."""
    dims, mass = (4, 4, 4, 4), 0.2
    t = TABLES["hypercube"]
    u = synth.gauge_links(dims, 0.4, 8408)
    b = synth.gaussian_spinor(dims, 8409, nrhs=2)
    log(f"generic class solve inner={inner}")
    U = bri.bri_pack_links(dims, dev(u), bri.F64)
    hi = bri.Operator(bri.bri_build_transporters(dims, U, bri.F64, 80), coef=t)
    lo = bri.Operator(bri.bri_build_transporters(dims, U, inner, 80), coef=t) if inner else None
    p = bri.solve_params(tol=1e-10, inner_tol=1e-3, inner_prec=inner)
    X, info = bri.bri_solve_cgne_op(dims, hi, bri.bri_pack_spinor(dims, dev(b), bri.F64), mass, p, op_lo=lo)
    assert info["converged"] and max(info["true_residual"]) <= 1e-10
    xs = soa_to_canon(dims, X)
    for r in range(2):
        res = ultralocal.apply(u, xs[r], mass, t) - b[r]
        assert np.linalg.norm(res) / np.linalg.norm(b[r]) <= 2e-10


def test_table_rejections(bri):
    dims = (4, 4, 4, 4)
    U = bri.bri_pack_links(dims, dev(synth.gauge_links(dims, 0.3, 8410)), bri.F64)
    x = bri.bri_pack_spinor(dims, dev(synth.gaussian_spinor(dims, 8411, nrhs=1)), bri.F64)
    W80 = bri.bri_build_transporters(dims, U, bri.F64, 80)
    bad = list(bri.TABLE_WILSON)
    bad[6] = float("nan")
    with pytest.raises(bri.BriError, match="not finite"):
        bri.bri_apply_op(dims, bri.Operator(W80, coef=bad), x, 0.1)
    with pytest.raises(ValueError, match="nine entries"):
        bri.Operator(W80, coef=(1.0, 2.0))
    # the inner operator of a mixed solve must carry the same table
    W32 = bri.bri_build_transporters(dims, U, bri.F32, 80)
    p = bri.solve_params(tol=1e-10, inner_tol=1e-3, inner_prec=bri.F32)
    with pytest.raises(bri.BriError, match="same coefficient table"):
        bri.bri_solve_cgne_op(dims, bri.Operator(W80, coef=bri.TABLE_WILSON), x, 0.1, p,
                              op_lo=bri.Operator(W32, coef=bri.TABLE_HYPERCUBE))


def test_overlap_with_hypercube_kernel(bri):
    """The overlap machinery takes any member: D_ov,m with the hypercube
    kernel against the exact dense overlap built on the oracle's kernel
    (rho = 0.5: at rho = 1 these links give the hypercube kernel a near-zero
    mode of gamma5 D(-rho))."""
    from oracle import overlap as oov
    dims, rho = (2, 2, 2, 2), 0.5
    t = TABLES["hypercube"]
    u = synth.gauge_links(dims, 0.5, 8412)
    dk = oov.kernel_matrix(u, rho, dense=ultralocal.dense_matrix(u, 0.0, t))
    ev = oov.ritz_reference(dk)
    lo, hi = 0.95 * ev[0], 1.05 * ev[-1]
    deg = next(d for d in (50, 100, 200, 400, 800, 1600) if oov.inv_sqrt_chebyshev(lo, hi, d)[1] < 1e-11)
    U = bri.bri_pack_links(dims, dev(u), bri.F64)
    op = bri.Operator(bri.bri_build_transporters(dims, U, bri.F64, 80), coef=t)
    psi = synth.gaussian_spinor(dims, 8413, nrhs=2)
    x = bri.bri_pack_spinor(dims, dev(psi), bri.F64)
    log(f"overlap with the hypercube kernel, degree {deg}")
    out, err = bri.bri_overlap_apply(dims, op, x, rho, 0.05, lo, hi, deg)
    assert err < 1e-11
    want = (oov.overlap_matrix(dk, rho, 0.05) @ psi.reshape(2, -1).T).T
    got = soa_to_canon(dims, out).reshape(2, -1)
    for r in range(2):
        assert np.linalg.norm(got[r] - want[r]) <= (2 * err + 1e-12) * np.linalg.norm(psi[r])


def test_table_fullsize_sampled(bri):
    """32^3 x 64 (the benchmark's lattice and launch): the hypercube column
    with FP32 and FP64 stored transporters, D and D^dag, on 64 random sites
    plus corners computed site by site by the oracle."""
    import torch
    dims, mass, t = (32, 32, 32, 64), 0.1, TABLES["hypercube"]
    u = synth.gauge_links(dims, 0.3, 4001)
    psi = synth.gaussian_spinor(dims, 4002, nrhs=1)
    rng = np.random.default_rng(8414)
    sites = np.concatenate([np.stack([rng.integers(0, L, 64) for L in dims], axis=1),
                            np.array([[0, 0, 0, 0], [31, 31, 31, 63], [0, 31, 0, 63]])])
    ref = ultralocal.apply_at(u, psi[0], mass, t, sites)
    # D^dag = gamma5 D gamma5 for every member of the class (pinned in the oracle tests)
    g5 = gamma5()
    p5 = np.einsum("st,...tc->...sc", g5, psi[0])
    ref_dag = np.einsum("st,ntc->nsc", g5, ultralocal.apply_at(u, p5, mass, t, sites))
    U = bri.bri_pack_links(dims, dev(u), bri.F64)
    for p in (1, 0):
        log(f"generic class fullsize prec={p}")
        op = bri.Operator(bri.bri_build_transporters(dims, U, p, 80), coef=t)
        x = bri.bri_pack_spinor(dims, dev(psi), p)
        for dag, want in ((False, ref), (True, ref_dag)):
            out = bri.bri_unpack_spinor(dims, bri.bri_apply_op(dims, op, x, mass, dagger=dag)).cpu().numpy()[0]
            got = np.stack([out[tt, z, y, xx] for xx, y, z, tt in sites])
            assert rel(got, want) <= TOL[p], (p, dag)
        del op, x
        torch.cuda.empty_cache()
