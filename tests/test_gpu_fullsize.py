"""Parity at the full benchmark sizes, in the launch configuration the
benchmark times (stored transporters, LDS-tiled kernel, one right-hand side;
at 32^3 x 64 the 32x16 tile for FP32 and FP64 with 80 offsets), on outputs
the oracle computes site by site: 256 random sites plus three corners of
32^3 x 64 and 24^3 x 48, for every stored precision and both transporter
stores, D and D^dag (the oracle's D^dag from D(y,x)^dag), and for the
recompute variant.  Each case is checked in the 2-norm over the sampled
outputs and element by element against the largest sampled element."""
import numpy as np
import pytest

import synth
from oracle import dirac
from tests.helpers import dev, log

pytestmark = pytest.mark.gpu

TOL = {(0, 0): 1e-12, (1, 1): 1e-5, (2, 1): 5e-3, (2, 2): 5e-3}
_inputs = {}


def inputs(dims, eps, seed):
    key = (dims, eps, seed)
    if key not in _inputs:
        _inputs.clear()
        u = synth.gauge_links(dims, eps, seed)
        psi = synth.gaussian_spinor(dims, seed + 1, nrhs=1)
        rng = np.random.default_rng(seed + 2)
        sites = np.stack([rng.integers(0, L, 256) for L in dims], axis=1)
        # include the lattice corners (every wrap-around direction)
        corners = np.array([[0, 0, 0, 0], [dims[0] - 1, dims[1] - 1, dims[2] - 1, dims[3] - 1],
                            [0, dims[1] - 1, 0, dims[3] - 1]])
        sites = np.concatenate([sites, corners])
        ref = dirac.apply_at(u, psi[0], 0.1, sites)
        refd = dirac.apply_dag_at(u, psi[0], 0.1, sites)
        _inputs[key] = (u, psi, sites, ref, refd)
    return _inputs[key]


def sampled(bri, dims, out, sites):
    got = bri.bri_unpack_spinor(dims, out).cpu().numpy()[0]
    return np.stack([got[t, z, y, x] for x, y, z, t in sites])


def check(got, ref, tol, what):
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    emax = float(np.abs(got - ref).max() / np.abs(ref).max())
    assert err <= tol and emax <= tol, f"{what}: rel {err:.3e} max-elem {emax:.3e} > {tol}"


@pytest.mark.parametrize("dims,eps,seed", [((32, 32, 32, 64), 0.3, 4001), ((24, 24, 24, 48), 0.4, 3001)])
def test_fullsize_sampled_parity(dims, eps, seed):
    import torch
    import paper_1012_3615_amd as bri
    u, psi, sites, ref, refd = inputs(dims, eps, seed)
    bri.bri_clear_apply_configs()
    U = bri.bri_pack_links(dims, dev(u), bri.F64)
    for wp, sp, noff in [(1, 1, 80), (1, 1, 40), (0, 0, 80), (2, 1, 80), (2, 2, 80)]:
        log(f"fullsize {dims} w={wp} s={sp} noff={noff} kernel={bri.bri_get_apply_config(dims, wp, sp, noff, 1)}")
        W = bri.bri_build_transporters(dims, U, wp, noff)
        x = bri.bri_pack_spinor(dims, dev(psi), sp)
        check(sampled(bri, dims, bri.bri_apply(dims, W, x, 0.1), sites), ref, TOL[(wp, sp)],
              f"D w={wp} s={sp} noff={noff}")
        check(sampled(bri, dims, bri.bri_apply_dag(dims, W, x, 0.1), sites), refd, TOL[(wp, sp)],
              f"D^dag w={wp} s={sp} noff={noff}")
        del W, x
        torch.cuda.empty_cache()
    log(f"fullsize {dims} recompute f32")
    U32 = bri.bri_pack_links(dims, dev(u), bri.F32)
    x = bri.bri_pack_spinor(dims, dev(psi), bri.F32)
    check(sampled(bri, dims, bri.bri_apply(dims, U32, x, 0.1, variant=bri.RECOMPUTE), sites), ref, 1e-5,
          "recompute D")
    check(sampled(bri, dims, bri.bri_apply_dag(dims, U32, x, 0.1, variant=bri.RECOMPUTE), sites), refd, 1e-5,
          "recompute D^dag")


def test_fullsize_mfma_12rhs_sampled():
    """The matrix-core apply at 32^3 x 64 in the launch the benchmark times
    (12 right-hand sides in one workgroup column, t chunks of 64, FP16
    store from the FP32 80-offset store): twelve Gaussian columns, D and
    D^dag at the sampled sites, each column within 5e-3 of the oracle in the
    2-norm and 1e-2 per element against its largest sampled element (the
    bars of the small-lattice matrix-core tests)."""
    import torch
    import paper_1012_3615_amd as bri
    dims, eps, seed = (32, 32, 32, 64), 0.3, 4001
    u, _, sites, _, _ = inputs(dims, eps, seed)
    V = int(np.prod(dims))
    idx = torch.as_tensor(sites[:, 0] + dims[0] * (sites[:, 1] + dims[1] * (sites[:, 2] + dims[2] * sites[:, 3])),
                          device="cuda")
    U = bri.bri_pack_links(dims, dev(u), bri.F64)
    Wm = bri.bri_pack_w_mfma(dims, bri.bri_build_transporters(dims, U, bri.F32, 80))
    del U
    x = torch.empty((12, 12, V, 2), dtype=torch.float32, device="cuda")
    refs, refds = [], []
    for r in range(12):
        log(f"fullsize mfma column {r}")
        psi = synth.gaussian_spinor(dims, seed + 10 + r, nrhs=1)
        refs.append(dirac.apply_at(u, psi[0], 0.1, sites).reshape(len(sites), 12))
        refds.append(dirac.apply_dag_at(u, psi[0], 0.1, sites).reshape(len(sites), 12))
        x[r] = bri.bri_pack_spinor(dims, dev(psi), bri.F32)[0]
        del psi
    xs, b2 = bri.bri_spinor_to_sites(dims, x, bound2=True)
    for dag, ref in ((False, refs), (True, refds)):
        log(f"fullsize mfma apply dagger={dag}")
        out = bri.bri_spinor_from_sites(dims, bri.bri_apply_mfma(dims, Wm, xs, 0.1, dagger=dag, bound2=b2))
        g = out[:, :, idx, :].double().cpu().numpy()  # [12 rhs, 12 comp, N, 2]
        g = g[..., 0] + 1j * g[..., 1]
        for r in range(12):
            got = g[r].T  # [N, 12]
            err = np.linalg.norm(got - ref[r]) / np.linalg.norm(ref[r])
            emax = float(np.abs(got - ref[r]).max() / np.abs(ref[r]).max())
            assert err <= 5e-3 and emax <= 1e-2, f"dagger={dag} rhs {r}: rel {err:.3e} max-elem {emax:.3e}"
        del out
