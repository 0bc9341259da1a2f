#!/usr/bin/env python3
"""Benchmark: Brillouin operator applications per second at 32^3 x 64.

One step = one application out = D_B psi of the 81-point Brillouin operator
(Eq. def_pref, c_SW = 0) on a 32^3 x 64 lattice, FP32 storage and FP32
arithmetic, with the 80 stored hypercube-averaged transporters (built once,
in FP64, before the timed region).  Inputs are seeded synthetic fields
resident in HBM: SU(3) links U = exp(i 0.3 H) (seed 4001), Gaussian spinor
(seed 4002), m = 0.1.

Printed (one JSON line): applications/s, the roofline of the apply kernel
(algorithmic bytes per launch over its mean launch time, measured with HIP
events on the library's stream), the CPU oracle timed on a bounded sample of
the same workload, and side measurements of the other variants.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline] [--cpu-full]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

DIMS = (32, 32, 32, 64)
MASS = 0.1
EPS = 0.3
SEED_U, SEED_PSI = 4001, 4002
HBM_PEAK_GBS = 8000.0
FLOPS_PER_SITE = 35376           # nominal flops per site and right-hand side
FP64_PEAK_TFS = 78.6
# relative residual each inner cycle of a mixed solve aims at: with 3e-4 the
# solves to 1e-10 take three FP64 refinement cycles instead of four at 1e-3
# for the same inner iterations (32^3 x 64, 12 sources: 0.92 vs 0.97 s on the
# matrix cores, 1.93 vs 2.05 s with FP32 inner solves; 1e-4 costs more
# iterations and 3e-3 a fourth cycle)
INNER_TOL = 3e-4
# transporter build: FP64 links read once (4 x 9 x 16 B) + FP32 80-offset store
# written once (80 x 9 x 8 B); 104 FP64 3x3 complex products (216 flops each)
BUILD_BYTES_PER_SITE = 4 * 9 * 16 + 80 * 9 * 8
BUILD_FLOPS_PER_SITE = 104 * 216
# link gradient with the transporters given: links, FP64 40-offset
# transporters, chi and psi read once, the gradient written once
GRAD_BYTES_PER_SITE = 4 * 9 * 16 + 40 * 9 * 16 + 2 * 12 * 16 + 4 * 9 * 16
# matrix-core 12-RHS apply: the site-major FP16 store read once (80 x 9 x 4 B),
# 12 site-major FP32 spinors read and written once (2 x 12 x 12 x 8 B); per site 20
# reduction steps x 6 v_mfma_f32_16x16x32_f16 of 16 x 16 x 32 x 2 flops each
MFMA_BYTES_PER_SITE = 80 * 9 * 4 + 2 * 12 * 12 * 8
MFMA_ISSUED_FLOPS_PER_SITE = 20 * 6 * 16 * 16 * 32 * 2
FP16_PEAK_TFS = 2500.0
# the headline kernel and the launcher that picks its tile shape
KERNEL_SOURCES = ["paper_1012_3615_amd/csrc/common.h", "paper_1012_3615_amd/csrc/stencil.h",
                  "paper_1012_3615_amd/csrc/apply_tiled.h", "paper_1012_3615_amd/csrc/apply_launch.h"]
PMC_FILE = os.path.join(ROOT, "profiles", "apply_tiled_f32_w80_32x32x32x64.pmc.json")


def bytes_per_site(n_off, wbytes, sbytes, nrhs=1):
    """Algorithmic HBM bytes per site: every stored transporter read once,
    each input spinor read once and each output spinor written once."""
    return n_off * 9 * wbytes + nrhs * 2 * 12 * sbytes


def kernel_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def timed_launches(torch, fn, steps, warmup):
    """Run fn warmup times, then time `steps` launches with one event pair per
    launch on the current stream (where the library launches).  Returns
    (total seconds, list of per-launch ms)."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    t0 = time.perf_counter()
    for s, e in ev:
        s.record()
        fn()
        e.record()
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    return total, [s.elapsed_time(e) for s, e in ev]


def batch_ms(torch, fn, steps, warmup, out=None):
    """Mean ms per launch of `steps` launches captured once in a HIP graph and
    replayed between one event pair: sub-millisecond kernels launched one by
    one from Python wait for the host (and an event pair per launch adds its
    own gap).  With `out`, the first and the last replay are checked against
    the eager result bit for bit."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ref = out.clone() if out is not None else None
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fn()
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        for _ in range(steps):
            fn()
    graph.replay()
    torch.cuda.synchronize()
    if ref is not None and not torch.equal(out, ref):
        raise RuntimeError("graph replay differs from the eager apply")
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(3):
        graph.replay()
    e.record()
    torch.cuda.synchronize()
    if ref is not None and not torch.equal(out, ref):
        raise RuntimeError("graph replay differs from the eager apply")
    return s.elapsed_time(e) / (3 * steps)


def cpu_baseline(u, psi, got, full=False):
    """The CPU oracle as it stands (plain numpy, FP64): the whole-field apply
    (oracle.dirac.apply: np.roll shifts, path-enumerated transporters, the
    direct 81-point sum) on seeded lattices of 4^4 and 8^4 (and 16^3 x 32 with
    full=True, about a minute per application), one warm-up then the median of
    three, with the BLAS thread pool open to every host core.  The value is
    the per-site rate of the largest lattice timed, in applications/s of the
    32^3 x 64 lattice.  The threads the oracle actually used are measured as
    process CPU time over wall time (numpy's per-site 3x3 products and
    einsum loops run on one thread whatever the BLAS setting).  Also the
    relative error of the timed GPU output `got` (canonical layout) at 64
    random sites against the pointwise oracle.  Returns (baseline dict, spot
    error)."""
    import numpy as np
    from threadpoolctl import threadpool_info, threadpool_limits
    import synth
    from oracle import dirac
    V = int(np.prod(DIMS))
    rs = np.random.default_rng(5)
    spot = np.stack([rs.integers(0, L, 64) for L in DIMS], axis=1)
    ref = dirac.apply_at(u, psi, MASS, spot)
    gs = np.stack([got[t, z, y, x] for x, y, z, t in spot])
    spot_err = float(np.linalg.norm(gs - ref) / np.linalg.norm(ref))
    ncpu = os.cpu_count() or 1
    sizes = [(4, 4, 4, 4), (8, 8, 8, 8)] + ([(16, 16, 16, 32)] if full else [])
    per_size = {}
    with threadpool_limits(limits=ncpu):
        blas = sorted({(p.get("internal_api"), p.get("num_threads")) for p in threadpool_info()})
        for dims in sizes:
            uu = synth.gauge_links(dims, EPS, SEED_U)
            pp = synth.gaussian_spinor(dims, SEED_PSI, nrhs=1)[0]
            dirac.apply(uu, pp, MASS)  # warm-up
            walls, cpus = [], []
            for _ in range(3):
                t0, c0 = time.perf_counter(), time.process_time()
                dirac.apply(uu, pp, MASS)
                walls.append(time.perf_counter() - t0)
                cpus.append(time.process_time() - c0)
            wall = float(np.median(walls))
            vs = int(np.prod(dims))
            per_size["x".join(map(str, dims))] = {
                "median_s": wall, "applies_s": 1.0 / wall, "sites_per_s": vs / wall,
                "gflops": FLOPS_PER_SITE * vs / wall / 1e9, "cpu_over_wall": float(sum(cpus) / sum(walls))}
    last = per_size["x".join(map(str, sizes[-1]))]
    used = max(1, int(round(max(e["cpu_over_wall"] for e in per_size.values()))))
    single = {"value": last["sites_per_s"] / V, "cores": used,
              "threads_used": f"process CPU time / wall time = {max(e['cpu_over_wall'] for e in per_size.values()):.2f}"}
    # the host's throughput: one oracle process per core of the GPU's CPU share
    # (at most 16), each timing three 8^4 applications after a warm-up, all
    # released together; the rate is the parent's count of applications over
    # the wall time of the whole concurrent window
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = ncpu
    nproc = max(1, min(16, avail))
    multi = cpu_throughput(nproc, 8)
    value = multi["sites_per_s"] / V if multi else single["value"]
    return {"value": value, "unit": "applies/s", "cores": nproc if multi else used, "kind": "oracle",
            "sample": (f"whole-field FP64 numpy oracle (oracle.dirac.apply), unmodified: {nproc} concurrent "
                       f"processes (one BLAS/OpenMP thread each) on 8x8x8x8 lattices (links exp(i {EPS} H)), "
                       f"three applications each after a warm-up, released together; value = sites per second "
                       f"of the whole window scaled to the 32x32x32x64 volume; single-process timings at "
                       f"{', '.join('x'.join(map(str, d)) for d in sizes)} (median of 3) under 'single_process'"),
            "host_cpu_count": ncpu, "cpu_affinity": avail, "blas_threads": [list(b) for b in blas],
            "multi_process": multi, "single_process": single, "sizes": per_size}, spot_err


def cpu_worker(L):
    """One oracle process of the throughput leg: inputs and a warm-up, then
    'ready'; on a line from the parent, three timed applications on L^4."""
    import numpy as np
    import synth
    from oracle import dirac
    dims = (L, L, L, L)
    uu = synth.gauge_links(dims, EPS, SEED_U)
    pp = synth.gaussian_spinor(dims, SEED_PSI, nrhs=1)[0]
    dirac.apply(uu, pp, MASS)
    print("ready", flush=True)
    sys.stdin.readline()
    walls = []
    for _ in range(3):
        t0 = time.perf_counter()
        dirac.apply(uu, pp, MASS)
        walls.append(time.perf_counter() - t0)
    print(json.dumps({"walls": walls}), flush=True)


def cpu_throughput(nproc, L):
    """Runs nproc cpu_worker processes (this file with --cpu-worker L) and
    returns the aggregate rate, or None if a worker failed."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    procs = [subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-worker", str(L)],
                              stdin=subprocess.PIPE, stdout=subprocess.PIPE, text=True, env=env)
             for _ in range(nproc)]
    try:
        if any(p.stdout.readline().strip() != "ready" for p in procs):
            return None
        t0 = time.perf_counter()
        for p in procs:
            p.stdin.write("go\n")
            p.stdin.flush()
        res = [json.loads(p.stdout.readline()) for p in procs]
        window = time.perf_counter() - t0
    finally:
        for p in procs:
            try:
                p.stdin.close()
            except OSError:
                pass
            try:
                p.wait(timeout=120)
            except subprocess.TimeoutExpired:
                p.kill()
                p.wait()
    vs = L ** 4
    applies = sum(len(r["walls"]) for r in res)
    per = sorted(w for r in res for w in r["walls"])
    return {"processes": nproc, "lattice": [L] * 4, "window_s": window, "applications": applies,
            "sites_per_s": applies * vs / window, "median_application_s": per[len(per) // 2],
            "gflops": FLOPS_PER_SITE * applies * vs / window / 1e9}


def traffic_from_profile(launch_bytes_alg):
    if not os.path.exists(PMC_FILE):
        return None
    with open(PMC_FILE) as f:
        p = json.load(f)
    if p.get("kernel_hash") != kernel_hash():
        return None
    return p.get("hbm_bytes_per_launch")


def solve_comparison(torch, bri, U64, dev, tol=1e-10):
    """Propagator solve: the 12 spin-colour point sources at the origin, to a
    true FP64 relative residual of 1e-10, (a) batched mixed precision (FP32
    inner CGNE with FP32 transporters, FP64 defect correction) against (b)
    twelve plain FP64 CGNE solves one after the other and (c) one plain FP64
    CGNE solve of the twelve sources batched.  Every solve checks its
    convergence after each iteration (a host read of the per-RHS state, tens
    of microseconds against ~17 ms per iteration), so none overshoots; the
    FP16-transporter inner solves aim at INNER_TOL per cycle like the FP32 one."""
    import numpy as np
    import synth
    src = synth.point_sources(DIMS)
    b = bri.bri_pack_spinor(DIMS, torch.from_numpy(src).to(dev), bri.F64)
    del src
    W64 = bri.bri_build_transporters(DIMS, U64, bri.F64, 80)
    W32 = bri.bri_build_transporters(DIMS, U64, bri.F32, 80)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p = bri.solve_params(tol=tol, inner_prec=bri.F32, inner_tol=INNER_TOL, check_every=1)
    _, im = bri.bri_solve_cgne(DIMS, W64, b, MASS, p, W_lo=W32)
    torch.cuda.synchronize()
    t_mixed = time.perf_counter() - t0
    # the same batched FP32 solve with FP64 refinement stopped at 1e-8
    t0 = time.perf_counter()
    p = bri.solve_params(tol=1e-8, inner_prec=bri.F32, inner_tol=INNER_TOL, check_every=1)
    _, i8 = bri.bri_solve_cgne(DIMS, W64, b, MASS, p, W_lo=W32)
    torch.cuda.synchronize()
    t_mixed8 = time.perf_counter() - t0
    del W32
    W16 = bri.bri_build_transporters(DIMS, U64, bri.F16, 80)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p = bri.solve_params(tol=tol, inner_prec=bri.F16, inner_tol=INNER_TOL, check_every=1)
    _, ih = bri.bri_solve_cgne(DIMS, W64, b, MASS, p, W_lo=W16)
    torch.cuda.synchronize()
    t_half = time.perf_counter() - t0
    del W16
    # the FP16-transporter inner solve with the matrix-core apply
    Wm = bri.bri_pack_w_mfma(DIMS, W64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p = bri.solve_params(tol=tol, inner_prec=bri.F16, inner_tol=INNER_TOL, check_every=1, inner_mfma=True)
    _, imf = bri.bri_solve_cgne(DIMS, W64, b, MASS, p, W_lo=Wm)
    torch.cuda.synchronize()
    t_mfma = time.perf_counter() - t0
    del Wm
    # plain FP64 CGNE with the twelve sources batched (one fused FP64 apply per step)
    t0 = time.perf_counter()
    p = bri.solve_params(tol=tol, inner_prec=bri.F64, check_every=1)
    _, ib = bri.bri_solve_cgne(DIMS, W64, b, MASS, p)
    torch.cuda.synchronize()
    t_batched = time.perf_counter() - t0
    t0 = time.perf_counter()
    iters, worst = 0, 0.0
    for r in range(12):
        _, ip = bri.bri_solve_cgne(DIMS, W64, b[r:r + 1].contiguous(), MASS, p)
        iters += ip["iterations"]
        worst = max(worst, ip["true_residual"][0])
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    return {"tol": tol, "mixed_s": t_mixed, "plain_fp64_12x_s": t_plain,
            "mixed_tol_1e-8_s": t_mixed8, "mixed_tol_1e-8_iterations": i8["iterations"],
            "mixed_tol_1e-8_max_true_residual": max(i8["true_residual"][:12]),
            "ratio_mixed_over_plain": t_mixed / t_plain,
            "mixed_iterations": im["iterations"], "mixed_outer": im["outer"],
            "mixed_max_true_residual": max(im["true_residual"][:12]),
            "mixed_f16w_s": t_half, "ratio_mixed_f16w_over_plain": t_half / t_plain,
            "mixed_f16w_iterations": ih["iterations"], "mixed_f16w_outer": ih["outer"],
            "mixed_f16w_max_true_residual": max(ih["true_residual"][:12]),
            "plain_iterations_total": iters, "plain_max_true_residual": worst,
            "plain_fp64_batched_s": t_batched, "plain_fp64_batched_iterations": ib["iterations"],
            "plain_fp64_batched_max_true_residual": max(ib["true_residual"][:12]),
            "ratio_mixed_over_plain_batched": t_mixed / t_batched,
            "ratio_mixed_f16w_over_plain_batched": t_half / t_batched,
            "mixed_f16w_mfma_s": t_mfma, "ratio_mixed_f16w_mfma_over_plain": t_mfma / t_plain,
            "ratio_mixed_f16w_mfma_over_plain_batched": t_mfma / t_batched,
            "mixed_f16w_mfma_iterations": imf["iterations"], "mixed_f16w_mfma_outer": imf["outer"],
            "mixed_f16w_mfma_max_true_residual": max(imf["true_residual"][:12])}


def solve_24x48(torch, bri, dev, tol=1e-10):
    """24^3 x 48, links eps 0.4 (seed 3001), Gaussian right-hand side (seed
    3002), m in {0.05, 0.2, 0.5}: mixed precision (FP32 or FP16 transporters,
    inner cycles to INNER_TOL) against plain FP64 CGNE, all to a true FP64 residual
    of 1e-10, every solve checking its convergence after each iteration."""
    import synth
    dims = (24, 24, 24, 48)
    u = synth.gauge_links(dims, 0.4, 3001)
    U = bri.bri_pack_links(dims, torch.from_numpy(u).to(dev), bri.F64)
    del u
    b = bri.bri_pack_spinor(dims, torch.from_numpy(synth.gaussian_spinor(dims, 3002, 1)).to(dev), bri.F64)
    W64 = bri.bri_build_transporters(dims, U, bri.F64, 80)
    Wlo = {bri.F32: bri.bri_build_transporters(dims, U, bri.F32, 80),
           bri.F16: bri.bri_build_transporters(dims, U, bri.F16, 80)}
    out = {}
    for m in (0.05, 0.2, 0.5):
        row = {}
        for name, prec, itol in (("plain_fp64", bri.F64, 0.5), ("mixed_f32", bri.F32, INNER_TOL),
                                 ("mixed_f16w", bri.F16, INNER_TOL)):
            p = bri.solve_params(tol=tol, inner_prec=prec, inner_tol=itol, check_every=1)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, info = bri.bri_solve_cgne(dims, W64, b, m, p, W_lo=Wlo.get(prec))
            torch.cuda.synchronize()
            row[name] = {"s": time.perf_counter() - t0, "iterations": info["iterations"],
                         "outer": info["outer"], "applies": info["applies"],
                         "true_residual": info["true_residual"][0]}
        for name in ("mixed_f32", "mixed_f16w"):
            row[name]["speedup_vs_plain"] = row["plain_fp64"]["s"] / row[name]["s"]
        out[f"m={m}"] = row
    return out


def variants_16_32(torch, bri, dev, steps=100):
    """The 16^3 x 32 lattice (links eps 0.3, seed 2001; Gaussian spinor, seed
    2002): 100 back-to-back applications each of the stored (W80 and W40) and
    the recompute variants in FP64 and FP32, one right-hand side, captured
    in a HIP graph and timed on its replays."""
    import numpy as np
    import synth
    dims = (16, 16, 16, 32)
    V = bri.volume(dims)
    u = torch.from_numpy(synth.gauge_links(dims, EPS, 2001)).to(dev)
    psi = torch.from_numpy(synth.gaussian_spinor(dims, 2002, 1)).to(dev)
    U64 = bri.bri_pack_links(dims, u, bri.F64)
    out = {}
    for prec, cb in ((bri.F64, 16), (bri.F32, 8)):
        x = bri.bri_pack_spinor(dims, psi, prec)
        name = "f64" if prec == bri.F64 else "f32"
        for noff in (80, 40):
            W = bri.bri_build_transporters(dims, U64, prec, noff)
            y = torch.empty_like(x)
            ms = batch_ms(torch, lambda: bri.bri_apply(dims, W, x, MASS, out=y), steps, 10, out=y)
            byts = bytes_per_site(noff, cb, cb) * V
            out[f"stored_w{noff}_{name}"] = {"ms": ms, "applies_s": 1e3 / ms,
                                             "gflops": FLOPS_PER_SITE * V / (ms * 1e-3) / 1e9,
                                             "alg_GBs": byts / (ms * 1e-3) / 1e9,
                                             "hbm_frac": byts / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
            del W
        Ux = U64 if prec == bri.F64 else bri.bri_pack_links(dims, u, bri.F32)
        y = torch.empty_like(x)
        ms = batch_ms(torch, lambda: bri.bri_apply(dims, Ux, x, MASS, variant=bri.RECOMPUTE, out=y), steps, 10,
                      out=y)
        out[f"recompute_{name}"] = {"ms": ms, "applies_s": 1e3 / ms,
                                    "gflops": FLOPS_PER_SITE * V / (ms * 1e-3) / 1e9}
    return out


def wilson_comparison(torch, bri, u, x32, W, dev, steps=50):
    """The Wilson operator (the paper's comparison operator, applied from the
    links, half-spinor hops) on the same 32^3 x 64 links and spinor, FP32
    and FP64, one right-hand side; `steps` applications captured in a HIP
    graph and timed on its replays.  The ratio of the headline Brillouin
    launch to the FP32 Wilson launch is the cost of one D_B application in
    Wilson applications on this GPU (the paper's conjecture: near 1 where
    both are bound by memory traffic); both sides are timed the same way, on
    graph replays (the Brillouin side with 20 applications per replay).  Algorithmic bytes per site: the four
    links of the site plus the spinor read and written (each neighbour
    spinor and backward link counted once, at its own site)."""
    import numpy as np
    V = int(np.prod(DIMS))
    out = {}
    for prec, cb, name in ((bri.F32, 8, "f32"), (bri.F64, 16, "f64")):
        U = bri.bri_pack_links(DIMS, torch.from_numpy(u).to(dev), prec)
        x = x32 if prec == bri.F32 else bri.bri_pack_spinor(DIMS, bri.bri_unpack_spinor(DIMS, x32), bri.F64)
        y = torch.empty_like(x)
        ms = batch_ms(torch, lambda: bri.bri_apply_wilson(DIMS, U, x, MASS, out=y), steps, 10, out=y)
        bps = 36 * cb + 24 * cb
        out[f"wilson_{name}"] = {"ms": ms, "applies_s": 1e3 / ms, "alg_bytes_per_site": bps,
                                 "alg_GBs": bps * V / (ms * 1e-3) / 1e9,
                                 "hbm_frac": bps * V / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
        del U, x, y
    yb = torch.empty_like(x32)
    b_ms = batch_ms(torch, lambda: bri.bri_apply(DIMS, W, x32, MASS, out=yb), 20, 5, out=yb)
    out["brillouin_f32_graph_ms"] = b_ms
    out["brillouin_f32_over_wilson_f32"] = b_ms / out["wilson_f32"]["ms"]
    return out


def wilson_brillouin_iterations(torch, bri, dev, tol=1e-10, k=200):
    """Inversion cost of the two operators at matched low end (Sec. 6 and its
    footnote: at a fixed pion mass the smallest eigenvalues of D^dag D are
    about equal, the largest near 2.5^2 for Brillouin and 7.5^2 for Wilson,
    so CG should need about a third of the iterations).  On the 16^3 x 32
    links (eps 0.3, seed 2001) the Wilson mass is tuned so that the smallest
    Ritz value of D_W^dag D_W (k Lanczos steps from a Gaussian start, seed
    2003) matches that of D_B^dag D_B at m_B; then plain FP64 CGNE to 1e-10
    from a Gaussian source (seed 2002) with each operator.  Wilson runs
    through the generic-class table: the same solver and transporter store,
    so the iteration counts compare the operators, not the kernels."""
    import numpy as np
    import synth
    dims = (16, 16, 16, 32)
    U = bri.bri_pack_links(dims, torch.from_numpy(synth.gauge_links(dims, EPS, 2001)).to(dev), bri.F64)
    W = bri.bri_build_transporters(dims, U, bri.F64, 80)
    ops = {"brillouin": bri.Operator(W), "wilson": bri.Operator(W, coef=bri.TABLE_WILSON)}
    b = bri.bri_pack_spinor(dims, torch.from_numpy(synth.gaussian_spinor(dims, 2002, 1)).to(dev), bri.F64)
    v0 = bri.bri_pack_spinor(dims, torch.from_numpy(synth.gaussian_spinor(dims, 2003, 1)).to(dev), bri.F64)

    def extremes(op, m):
        a, bb, _ = bri.bri_lanczos(dims, op, m, k, v0)
        r = bri.bri_ritz_values(a, bb)
        return float(r[0]), float(r[-1])

    def cgne(op, m):
        _, info = bri.bri_solve_cgne_op(dims, op, b, m, bri.solve_params(tol=tol, inner_prec=bri.F64))
        return int(info["iterations"]), float(info["true_residual"][0])

    out = {}
    for m_b in (0.05, 0.2):
        lo_b, hi_b = extremes(ops["brillouin"], m_b)
        m_w = m_b
        for _ in range(4):  # sqrt(lambda_min) grows about one for one with m
            lo_w, _ = extremes(ops["wilson"], m_w)
            m_w += float(np.sqrt(lo_b) - np.sqrt(lo_w))
        lo_w, hi_w = extremes(ops["wilson"], m_w)
        it_b, res_b = cgne(ops["brillouin"], m_b)
        it_w, res_w = cgne(ops["wilson"], m_w)
        out[f"m_B={m_b}"] = {
            "m_W": m_w, "lambda_min_B": lo_b, "lambda_min_W": lo_w, "lambda_max_B": hi_b, "lambda_max_W": hi_w,
            "condition_B": hi_b / lo_b, "condition_W": hi_w / lo_w,
            "cgne_iterations_B": it_b, "cgne_iterations_W": it_w, "iterations_B_over_W": it_b / it_w,
            "sqrt_condition_ratio": float(np.sqrt((hi_b / lo_b) / (hi_w / lo_w))),
            "true_residual_B": res_b, "true_residual_W": res_w}
    return out


def gradient_timing(torch, bri, dev):
    """FP64 link gradient of S = Re<chi, D psi> at 16^3 x 32 (the gradient
    lattice), as the autograd Function runs it: forward = transporter build
    (80 offsets) + apply; backward = one FP64 40-offset transporter build
    shared by apply_dag (psi gradient) and the link gradient."""
    import synth
    import numpy as np
    dims = (16, 16, 16, 32)
    u = synth.gauge_links(dims, EPS, 5101)
    U = bri.bri_pack_links(dims, torch.from_numpy(u).to(dev), bri.F64)
    chi = bri.bri_pack_spinor(dims, torch.from_numpy(synth.gaussian_spinor(dims, 5103, 1)).to(dev), bri.F64)
    psi = bri.bri_pack_spinor(dims, torch.from_numpy(synth.gaussian_spinor(dims, 5104, 1)).to(dev), bri.F64)

    def fwd():
        W = bri.bri_build_transporters(dims, U, bri.F64, 80)
        return bri.bri_apply(dims, W, psi, MASS)

    def bwd():
        W40 = bri.bri_build_transporters(dims, U, bri.F64, 40)
        bri.bri_apply_dag(dims, W40, chi, MASS)
        return bri.bri_grad_links(dims, U, chi, psi, W40=W40)

    _, pf = timed_launches(torch, fwd, 5, 2)
    _, pb = timed_launches(torch, bwd, 5, 2)
    tf, tb = float(np.mean(pf)), float(np.mean(pb))
    # the link gradient alone (bri_grad_links_w, FP64 40-offset transporters
    # given): it must read the links, the transporters, chi and psi once and
    # write the gradient once
    V = bri.volume(dims)
    W40 = bri.bri_build_transporters(dims, U, bri.F64, 40)
    _, pg = timed_launches(torch, lambda: bri.bri_grad_links(dims, U, chi, psi, W40=W40), 5, 2)
    tg = float(np.mean(pg))
    gbps = GRAD_BYTES_PER_SITE * V / (tg * 1e-3) / 1e9
    return {"forward_ms": tf, "backward_ms": tb, "backward_over_forward": tb / tf,
            "grad_links_w": {"ms": tg, "alg_bytes_per_site": GRAD_BYTES_PER_SITE, "alg_GBs": gbps,
                             "hbm_frac": gbps / HBM_PEAK_GBS, "bound": "hbm",
                             "kernels": "k_grad_fused + k_grad_gather"}}


def build_roofline(torch, bri, U64, steps=3):
    """The transporter build at 32^3 x 64 into the FP32 80-offset store (the
    headline's transporters), timed with HIP events on the library's stream.
    Algorithmic bytes per site: the FP64 links read once and the FP32 store
    written once; flops: the 104 FP64 3x3 complex products of the hop-order
    recursion over the 40 canonical offsets (12 two-hop x 2, 16 three-hop
    x 3, 8 four-hop x 4; the 1-hop transporters are the links)."""
    import numpy as np
    V = bri.volume(DIMS)
    W = bri.bri_build_transporters(DIMS, U64, bri.F32, 80)
    _, p = timed_launches(torch, lambda: bri.bri_build_transporters(DIMS, U64, bri.F32, 80, out=W), steps, 1)
    ms = float(np.mean(p))
    del W
    gbps = BUILD_BYTES_PER_SITE * V / (ms * 1e-3) / 1e9
    tfs = BUILD_FLOPS_PER_SITE * V / (ms * 1e-3) / 1e12
    return {"ms": ms, "alg_bytes_per_site": BUILD_BYTES_PER_SITE, "alg_GBs": gbps, "hbm_frac": gbps / HBM_PEAK_GBS,
            "flops_per_site": BUILD_FLOPS_PER_SITE, "fp64_TFs": tfs, "fp64_frac": tfs / FP64_PEAK_TFS,
            "bound": "hbm", "roofline_ms": max(BUILD_BYTES_PER_SITE * V / HBM_PEAK_GBS / 1e6,
                                               BUILD_FLOPS_PER_SITE * V / FP64_PEAK_TFS / 1e9),
            "kernels": "k_build_fused<float2, 80> (one launch)"}


def production_operator(torch, bri, U64, dev, psi, tol=1e-10):
    """The paper's production operator (Sec. 5) at 32^3 x 64: one APE step
    (alpha 0.72), transporters back-projected to SU(3) and stored as two rows,
    and the clover term (c_SW = 1).  Build times, apply times per form (HIP
    events per launch), and the 12-source propagator solve to a true FP64
    residual of 1e-10, mixed precision (FP32 or FP16 two-row transporters
    and FP32 clover inside) against twelve plain FP64 solves."""
    import numpy as np
    import synth
    V = bri.volume(DIMS)
    out = {}

    def timed(fn, steps=10, warm=2):
        _, p = timed_launches(torch, fn, steps, warm)
        return float(np.mean(p))

    out["ape_ms"] = timed(lambda: bri.bri_ape_smear(DIMS, U64, 0.72), 3, 1)
    Us = bri.bri_ape_smear(DIMS, U64, 0.72)
    out["build_su3_2row_f32_ms"] = timed(lambda: bri.bri_build_transporters_ex(DIMS, Us, bri.F32, 80,
                                                                               bri.W_SU3_2ROW), 3, 1)
    out["build_clover_f32_ms"] = timed(lambda: bri.bri_build_clover(DIMS, Us, 1.0, bri.F32), 3, 1)
    cb = {bri.F64: 16, bri.F32: 8, bri.F16: 4}
    xs = {sp: bri.bri_pack_spinor(DIMS, torch.from_numpy(psi).to(dev), sp) for sp in (bri.F32, bri.F64)}
    for name, wp, sp, form in (("su3_2row_clover_f32", bri.F32, bri.F32, bri.W_SU3_2ROW),
                               ("su3_full_clover_f32", bri.F32, bri.F32, bri.W_SU3),
                               ("su3_2row_clover_f16w_f32s", bri.F16, bri.F32, bri.W_SU3_2ROW),
                               ("su3_2row_clover_f64", bri.F64, bri.F64, bri.W_SU3_2ROW)):
        op = bri.Operator(bri.bri_build_transporters_ex(DIMS, Us, wp, 80, form), form,
                          bri.bri_build_clover(DIMS, Us, 1.0, sp))
        x = xs[sp]
        y = torch.empty_like(x)
        ms = timed(lambda: bri.bri_apply_op(DIMS, op, x, MASS, out=y), 20, 3)
        rows = 6 if form == bri.W_SU3_2ROW else 9
        byts = V * (80 * rows * cb[wp] + 2 * 12 * cb[sp] + 36 * cb[sp])
        out[name] = {"ms": ms, "applies_s": 1e3 / ms, "alg_bytes_per_site": byts // V,
                     "alg_GBs": byts / (ms * 1e-3) / 1e9, "hbm_frac": byts / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
        del op, y
        torch.cuda.empty_cache()
    del xs
    # propagator solve on the production operator
    src = synth.point_sources(DIMS)
    b = bri.bri_pack_spinor(DIMS, torch.from_numpy(src).to(dev), bri.F64)
    del src
    hi = bri.Operator(bri.bri_build_transporters_ex(DIMS, Us, bri.F64, 80, bri.W_SU3_2ROW), bri.W_SU3_2ROW,
                      bri.bri_build_clover(DIMS, Us, 1.0, bri.F64))
    lo = bri.Operator(bri.bri_build_transporters_ex(DIMS, Us, bri.F32, 80, bri.W_SU3_2ROW), bri.W_SU3_2ROW,
                      bri.bri_build_clover(DIMS, Us, 1.0, bri.F32))
    x12 = bri.bri_pack_spinor(DIMS, torch.from_numpy(synth.point_sources(DIMS)).to(dev), bri.F32)
    y12 = torch.empty_like(x12)
    out["su3_2row_clover_f32_12rhs_ms"] = timed(lambda: bri.bri_apply_op(DIMS, lo, x12, MASS, out=y12), 5, 2)
    del x12, y12
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p = bri.solve_params(tol=tol, inner_prec=bri.F32, inner_tol=1e-3, check_every=4)
    _, im = bri.bri_solve_cgne_op(DIMS, hi, b, MASS, p, op_lo=lo)
    torch.cuda.synchronize()
    t_mixed = time.perf_counter() - t0
    del lo
    lo16 = bri.Operator(bri.bri_build_transporters_ex(DIMS, Us, bri.F16, 80, bri.W_SU3_2ROW), bri.W_SU3_2ROW,
                        bri.bri_build_clover(DIMS, Us, 1.0, bri.F32))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p = bri.solve_params(tol=tol, inner_prec=bri.F16, inner_tol=1e-2, check_every=4)
    _, ih = bri.bri_solve_cgne_op(DIMS, hi, b, MASS, p, op_lo=lo16)
    torch.cuda.synchronize()
    t_half = time.perf_counter() - t0
    del lo16
    # plain FP64 CGNE with the twelve sources batched (one fused FP64 apply per step)
    t0 = time.perf_counter()
    p = bri.solve_params(tol=tol, inner_prec=bri.F64, check_every=4)
    _, ib = bri.bri_solve_cgne_op(DIMS, hi, b, MASS, p)
    torch.cuda.synchronize()
    t_batched = time.perf_counter() - t0
    t0 = time.perf_counter()
    iters, worst = 0, 0.0
    for r in range(12):
        _, ip = bri.bri_solve_cgne_op(DIMS, hi, b[r:r + 1].contiguous(), MASS, p)
        iters += ip["iterations"]
        worst = max(worst, ip["true_residual"][0])
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    out["solve_12rhs"] = {"tol": tol, "mixed_s": t_mixed, "plain_fp64_12x_s": t_plain,
                          "ratio_mixed_over_plain": t_mixed / t_plain, "mixed_iterations": im["iterations"],
                          "mixed_outer": im["outer"], "mixed_max_true_residual": max(im["true_residual"][:12]),
                          "mixed_f16w_s": t_half, "ratio_mixed_f16w_over_plain": t_half / t_plain,
                          "mixed_f16w_iterations": ih["iterations"], "mixed_f16w_outer": ih["outer"],
                          "mixed_f16w_max_true_residual": max(ih["true_residual"][:12]),
                          "plain_iterations_total": iters, "plain_max_true_residual": worst,
                          "plain_fp64_batched_s": t_batched, "plain_fp64_batched_iterations": ib["iterations"],
                          "plain_fp64_batched_max_true_residual": max(ib["true_residual"][:12]),
                          "ratio_mixed_over_plain_batched": t_mixed / t_batched,
                          "ratio_mixed_f16w_over_plain_batched": t_half / t_batched}
    return out


def overlap_kernel(torch, bri, dev):
    """The overlap kernel of Sec. 7 at 24^3 x 48 (links eps 0.4, seed 3001):
    the Brillouin operator with one APE step and SU(3) back-projected (two-row)
    transporters, c_SW = 0, at mass -rho, rho = 1.  300 Lanczos steps on
    D^dag D (three-term recurrence, spurious copies filtered) give the Ritz
    values of Sec. 7.3 (1st, 10th, largest); sign(H) is then applied to 1e-10
    on [0.9 r_1, 1.05 r_max] and timed."""
    import numpy as np
    import synth
    dims, rho = (24, 24, 24, 48), 1.0
    u = synth.gauge_links(dims, 0.4, 3001)
    U = bri.bri_pack_links(dims, torch.from_numpy(u).to(dev), bri.F64)
    del u
    Us = bri.bri_ape_smear(dims, U, 0.72)
    op = bri.Operator(bri.bri_build_transporters_ex(dims, Us, bri.F64, 80, bri.W_SU3_2ROW), bri.W_SU3_2ROW)
    del U, Us
    v0 = bri.bri_pack_spinor(dims, torch.from_numpy(synth.gaussian_spinor(dims, 3003, 1)).to(dev), bri.F64)
    k = 300
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    a, b, _ = bri.bri_lanczos(dims, op, -rho, k, v0)
    t_lanczos = time.perf_counter() - t0
    r = bri.bri_ritz_values(a, b)
    lo, hi = 0.9 * r[0], 1.05 * r[-1]
    deg = bri.sign_degree(lo, hi, 1e-10)
    out = torch.empty_like(v0)
    _, p = timed_launches(torch, lambda: bri.bri_sign_h(dims, op, -rho, v0, lo, hi, deg, out=out,
                                                        with_error=False), 3, 1)
    ms = float(np.mean(p))
    # low modes of H = gamma5 D(-rho) (kept-basis Lanczos + Rayleigh-Ritz, 160
    # FP64 basis fields = 20 GB) and the sign function deflated by them
    n_low, kl = 8, 160
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    vecs, ev, res = bri.bri_overlap_lowmodes(dims, op, -rho, kl, v0, n_low)
    torch.cuda.synchronize()
    t_low = time.perf_counter() - t0
    lo_d = 0.95 * float(r[n_low])
    deg_d = bri.sign_degree(lo_d, hi, 1e-10)
    _, p = timed_launches(torch, lambda: bri.bri_sign_h(dims, op, -rho, v0, lo_d, hi, deg_d, low_vecs=vecs,
                                                        low_evals=ev, out=out, with_error=False), 3, 1)
    ms_d = float(np.mean(p))
    # how far the deflated result is from the undeflated one (both on the GPU):
    # the deflation is only as exact as the modes' residuals
    ref = torch.empty_like(v0)
    bri.bri_sign_h(dims, op, -rho, v0, lo, hi, deg, out=ref, with_error=False)
    dev_defl = float(torch.linalg.vector_norm(out - ref) / torch.linalg.vector_norm(v0))
    del vecs, ref
    low = {"n_low": n_low, "lanczos_steps": kl, "s": t_low, "abs_evals_H": [float(abs(e)) for e in ev],
           "max_residual_norm": float(np.max(res)), "deflated_interval": [lo_d, hi],
           "deflated_degree_1e-10": deg_d, "deflated_sign_ms": ms_d,
           "deflated_minus_undeflated_rel": dev_defl}
    return {"lattice": list(dims), "kernel": "Brillouin, 1 APE step (0.72), SU(3) two-row W, c_SW = 0",
            "low_modes": low,
            "rho": rho, "lanczos_steps": k, "lanczos_s": t_lanczos, "ritz_kept": int(len(r)),
            "ritz_1st": float(r[0]), "ritz_10th": float(r[9]), "ritz_largest": float(r[-1]),
            "condition": float(r[-1] / r[0]), "condition_without_9_lowest": float(r[-1] / r[9]),
            "sign_interval": [lo, hi], "sign_degree_1e-10": deg,
            "sign_error_bound": bri.bri_sign_approx_error(lo, hi, deg),
            "sign_ms": ms, "ms_per_D_apply_in_sign": ms / (2 * deg + 3)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-full", action="store_true",
                    help="also time the whole-field oracle at 16^3x32 (about four minutes)")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--cpu-worker", type=int, default=0, help=argparse.SUPPRESS)
    a = ap.parse_args()
    if a.cpu_worker:
        cpu_worker(a.cpu_worker)
        return
    if a.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU only (asked for --gpus {a.gpus}); "
              "the multi-GPU decomposition is a design, not a measured path", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import synth
    import paper_1012_3615_amd as bri

    V = bri.volume(DIMS)
    t0 = time.perf_counter()
    u = synth.gauge_links(DIMS, EPS, SEED_U)
    psi = synth.gaussian_spinor(DIMS, SEED_PSI, nrhs=1)
    gen_s = time.perf_counter() - t0

    dev = torch.device("cuda:0")
    U64 = bri.bri_pack_links(DIMS, torch.from_numpy(u).to(dev), bri.F64)
    x32 = bri.bri_pack_spinor(DIMS, torch.from_numpy(psi).to(dev), bri.F32)
    torch.cuda.synchronize()
    tb = time.perf_counter()
    W = bri.bri_build_transporters(DIMS, U64, bri.F32, 80)
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - tb) * 1e3
    out = torch.empty_like(x32)

    # calibration copy of known size (for the PMC traffic scale factor)
    cal = torch.empty(256 << 20, dtype=torch.uint8, device=dev)
    cal2 = torch.empty_like(cal)
    cal2.copy_(cal)
    torch.cuda.synchronize()

    total_s, per = timed_launches(torch, lambda: bri.bri_apply(DIMS, W, x32, MASS, out=out),
                                  a.steps, a.warmup)
    per_ms = float(np.mean(per))
    value = a.steps / total_s
    bps = bytes_per_site(80, 8, 8)
    launch_bytes = bps * V
    achieved = launch_bytes / (per_ms * 1e-3) / 1e9

    # the timed output, kept for the spot parity check of the CPU-baseline leg
    got = bri.bri_unpack_spinor(DIMS, out).cpu().numpy()[0]

    # reference streams on the same GPU, measured after the timed region: a
    # device-wide read (torch sum over 8 GiB) and a 2 GiB copy (bytes read +
    # written), the achievable rates the headline is also priced against
    def stream_ms(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        e1.synchronize()
        return e0.elapsed_time(e1) / reps
    big = torch.ones(1 << 30, dtype=torch.float64, device=dev)
    read_gbs = big.numel() * 8 / stream_ms(lambda: big.sum()) / 1e6
    del big
    ca = torch.empty(1 << 31, dtype=torch.uint8, device=dev)
    cb = torch.empty_like(ca)
    copy_gbs = 2 * ca.numel() / stream_ms(lambda: cb.copy_(ca)) / 1e6
    del ca, cb
    torch.cuda.empty_cache()

    res = {
        "metric": "D_B applies/sec at 32^3x64 (FP32, stored 80 transporters)",
        "value": value,
        "unit": "applies/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": total_s / a.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "brillouin_apply_32x32x32x64", "lattice": list(DIMS),
                   "variant": "stored", "n_offsets": 80, "w_prec": "f32", "s_prec": "f32",
                   "nrhs": 1, "mass": MASS, "links": f"exp(i*{EPS}*H), seed {SEED_U}",
                   "spinor": f"gaussian, seed {SEED_PSI}"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic_from_profile(launch_bytes),
                     "kernel": "k_apply_tiled<80,float2,float2,float,false,32,16,1,true,true,3,false>",
                     "alg_bytes_per_site": bps, "alg_bytes_per_launch": launch_bytes,
                     "kernel_ms": per_ms,
                     # the same time priced at the minimum bytes of any stored scheme (W40)
                     "frac_vs_w40_min": bytes_per_site(40, 8, 8) * V / (per_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     # measured on this GPU after the timed region (see above)
                     "measured_read_GBs": read_gbs, "measured_copy_GBs": copy_gbs,
                     "frac_vs_measured_read": achieved / read_gbs, "frac_vs_measured_copy": achieved / copy_gbs},
        "gflops": FLOPS_PER_SITE * V / (per_ms * 1e-3) / 1e9,
        "build_transporters_ms": build_ms,  # first build, host clock (includes the first launches)
        "input_generation_s": gen_s,
    }

    if not a.no_extras:
        extras = {}

        def bench_variant(name, Wv, xv, n_off, wb, sb, variant=bri.STORED, dag=False, steps=20):
            fn = (lambda: bri.bri_apply_dag(DIMS, Wv, xv, MASS, variant=variant)) if dag else \
                 (lambda: bri.bri_apply(DIMS, Wv, xv, MASS, variant=variant))
            # ten warm-up launches: the GPU idles during the host-side parity check
            _, p = timed_launches(torch, fn, steps, 10)
            ms = float(np.mean(p))
            d = {"ms": ms, "applies_s": 1e3 / ms}
            if wb:
                byts = bytes_per_site(n_off, wb, sb, xv.shape[0]) * V
                d["alg_GBs"] = byts / (ms * 1e-3) / 1e9
                d["hbm_frac"] = d["alg_GBs"] / HBM_PEAK_GBS
                d["frac_vs_w40_min"] = bytes_per_site(40, wb, sb, xv.shape[0]) * V / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS
            extras[name] = d

        bench_variant("stored_w80_f32_dag", W, x32, 80, 8, 8, dag=True)
        # the same stored apply for other members of the generic class of
        # Sec. 8 (coefficients from a run-time table instead of constants)
        for tname, tab in (("hypercube", bri.TABLE_HYPERCUBE), ("wilson", bri.TABLE_WILSON)):
            opt = bri.Operator(W, coef=tab)
            _, p = timed_launches(torch, lambda: bri.bri_apply_op(DIMS, opt, x32, MASS, out=out), 20, 10)
            ms = float(np.mean(p))
            gbs = bytes_per_site(80, 8, 8) * V / (ms * 1e-3) / 1e9
            extras[f"table_{tname}_w80_f32"] = {"ms": ms, "applies_s": 1e3 / ms, "alg_GBs": gbs,
                                                "hbm_frac": gbs / HBM_PEAK_GBS}
        W40 = bri.bri_build_transporters(DIMS, U64, bri.F32, 40)
        bench_variant("stored_w40_f32", W40, x32, 40, 8, 8)
        del W40
        W16 = bri.bri_build_transporters(DIMS, U64, bri.F16, 80)
        bench_variant("stored_w80_f16w_f32s", W16, x32, 80, 4, 8)
        x16 = bri.bri_pack_spinor(DIMS, torch.from_numpy(psi).to(dev), bri.F16)
        bench_variant("stored_w80_f16w_f16s", W16, x16, 80, 4, 4)
        del W16, x16
        x64 = bri.bri_pack_spinor(DIMS, torch.from_numpy(psi).to(dev), bri.F64)
        W64 = bri.bri_build_transporters(DIMS, U64, bri.F64, 80)
        bench_variant("stored_w80_f64", W64, x64, 80, 16, 16)
        del W64
        U32 = bri.bri_pack_links(DIMS, torch.from_numpy(u).to(dev), bri.F32)
        bench_variant("recompute_f32", U32, x32, 0, 0, 0, variant=bri.RECOMPUTE, steps=5)
        bench_variant("recompute_f64", U64, x64, 0, 0, 0, variant=bri.RECOMPUTE, steps=5)
        del U32, x64
        # 12 spin-colour point sources in one fused launch, configuration from the autotuner
        from paper_1012_3615_amd import autotune
        src = synth.point_sources(DIMS)
        x12 = bri.bri_pack_spinor(DIMS, torch.from_numpy(src).to(dev), bri.F32)
        # (timed in this run, not read from a cache; the choice is installed
        # for the 12-RHS shape only and stays for the solves below)
        name, _, table, cached = autotune.tune(DIMS, W, x12, MASS, reps=3, use_cache=False)
        bench_variant("stored_w80_f32_12rhs", W, x12, 80, 8, 8, steps=5)
        extras["stored_w80_f32_12rhs"]["autotuned"] = name
        extras["stored_w80_f32_12rhs"]["autotune_ms"] = table
        extras["stored_w80_f32_12rhs"]["autotune_from_cache"] = cached
        # the same 12 sources on the matrix cores (FP16 operands, FP32
        # accumulation): the site-major FP16 store packed from the FP32 W80
        # and site-major FP32 spinors [V][12][12] (the conversions from and
        # to the SoA layout, which also give the per-source bounds, timed
        # on their own)
        Wm = bri.bri_pack_w_mfma(DIMS, W)
        xs, b2 = bri.bri_spinor_to_sites(DIMS, x12, bound2=True)
        o12 = torch.empty_like(xs)
        _, p = timed_launches(torch, lambda: bri.bri_apply_mfma(DIMS, Wm, xs, MASS, bound2=b2, out=o12), 5, 10)
        ms = float(np.mean(p))
        _, pb = timed_launches(torch, lambda: bri.bri_spinor_to_sites(DIMS, x12, out=o12, bound2=b2), 5, 3)
        _, pf = timed_launches(torch, lambda: bri.bri_spinor_from_sites(DIMS, xs, out=x12), 5, 3)
        byts = MFMA_BYTES_PER_SITE * V
        issued = MFMA_ISSUED_FLOPS_PER_SITE * V
        extras["mfma_w80_f16_12rhs"] = {
            "ms": ms, "applies_s": 1e3 / ms, "alg_GBs": byts / (ms * 1e-3) / 1e9,
            "hbm_frac": byts / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "mfma_issued_TFs": issued / (ms * 1e-3) / 1e12,
            "mfma_frac_fp16_dense": issued / (ms * 1e-3) / 1e12 / FP16_PEAK_TFS,
            "to_sites_with_bound_ms": float(np.mean(pb)), "from_sites_ms": float(np.mean(pf)),
            "kernel": "k_apply_mfma<3> (4x2 tile, 8 wavefronts, 12 rhs per workgroup, site-major spinors)"}
        del Wm, b2, o12, x12, xs
        x12 = bri.bri_pack_spinor(DIMS, torch.from_numpy(src).to(dev), bri.F64)
        W64 = bri.bri_build_transporters(DIMS, U64, bri.F64, 80)
        name, _, _, cached = autotune.tune(DIMS, W64, x12, MASS, reps=2, use_cache=False)
        bench_variant("stored_w80_f64_12rhs", W64, x12, 80, 16, 16, steps=3)
        extras["stored_w80_f64_12rhs"]["autotuned"] = name
        extras["stored_w80_f64_12rhs"]["autotune_from_cache"] = cached
        del x12, W64, src
        torch.cuda.empty_cache()
        res["extras"] = extras

    if not a.no_extras:
        res["build_transporters_32x32x32x64"] = build_roofline(torch, bri, U64)
        res["wilson_32x32x32x64"] = wilson_comparison(torch, bri, u, x32, W, dev)
    if not a.no_extras and not a.no_solve:
        res["solve_12rhs"] = solve_comparison(torch, bri, U64, dev)
    if not a.no_extras:
        res["variants_16x16x16x32"] = variants_16_32(torch, bri, dev)
        res["gradient_16x16x16x32"] = gradient_timing(torch, bri, dev)
        res["wilson_vs_brillouin_cgne_16x16x16x32"] = wilson_brillouin_iterations(torch, bri, dev)
    if not a.no_extras and not a.no_solve:
        res["solve_24x24x24x48"] = solve_24x48(torch, bri, dev)
    if not a.no_extras and not a.no_solve:
        del W, out
        torch.cuda.empty_cache()
        res["production_operator"] = production_operator(torch, bri, U64, dev, psi)
        torch.cuda.empty_cache()
        res["overlap_kernel_24x24x24x48"] = overlap_kernel(torch, bri, dev)

    if not a.no_cpu_baseline:
        res["cpu_baseline"], res["spot_parity_rel_err"] = cpu_baseline(u, psi[0], got, full=a.cpu_full)
    else:
        res["cpu_baseline"], res["spot_parity_rel_err"] = None, None
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
