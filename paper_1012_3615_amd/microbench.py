"""Microbenchmark of the operator variants (for timing and for rocprofv3).

    python -m paper_1012_3615_amd.microbench --dims 32 32 32 64 --reps 3 \\
        --variants tile_w80_f32 gather_w80_f32 tile_w40_f32 tile_w80_f16 \\
                   tile12_w80_f32 recompute_f32 stream

Each variant builds its inputs (links exp(i 0.3 H), seed 4001; Gaussian
spinors; the 12 point sources for the 12-RHS variant; for the production
operator forms prod*: one APE step, back-projected transporters whole or as
two rows, and the clover term; build_w80_f32: the transporter build into
the FP32 80-offset store; mfma12_w80_f16: the matrix-core apply of the 12
point sources; grad_w40: the link gradient with the FP64
40-offset transporters given; overlap_sign_24: sign(gamma5 D) at 24^3 x 48
to 1e-10 for the smeared, projected kernel at mass -1; wilson_f32/_f64: the
Wilson comparison operator from the links), runs one untimed
launch, then `reps` launches timed with HIP events on the current stream,
and prints one line per variant.  `stream` times a plain device read of a
8 GiB buffer (torch sum) and a 2 GiB copy, as a reference for the
achievable HBM bandwidth.  Inputs come from the seeded generator that runs
on the device, so large lattices start quickly.
"""
from __future__ import annotations

import argparse
import json

import torch

import synth
from . import api as bri

CB = {bri.F64: 16, bri.F32: 8, bri.F16: 4}

# name -> (variant, w_prec, s_prec, n_offsets, nrhs, kernel, rhs_per_thread)
VARIANTS = {
    "tile_w80_f32": (bri.STORED, bri.F32, bri.F32, 80, 1, 1, 1),
    "tile_w80_f32_dag": (bri.STORED, bri.F32, bri.F32, 80, 1, 1, 1),
    "gather_w80_f32": (bri.STORED, bri.F32, bri.F32, 80, 1, 0, 1),
    "tile_w40_f32": (bri.STORED, bri.F32, bri.F32, 40, 1, 1, 1),
    "tile_w80_f16": (bri.STORED, bri.F16, bri.F32, 80, 1, 1, 1),
    "tile_w80_f16h": (bri.STORED, bri.F16, bri.F16, 80, 1, 1, 1),
    "tile_w80_f64": (bri.STORED, bri.F64, bri.F64, 80, 1, 1, 1),
    "tile12_w80_f32": (bri.STORED, bri.F32, bri.F32, 80, 12, 1, 2),
    "tile12_w80_f16": (bri.STORED, bri.F16, bri.F32, 80, 12, 1, 1),
    "tile12_w80_f64": (bri.STORED, bri.F64, bri.F64, 80, 12, 1, 2),
    "recompute_f32": (bri.RECOMPUTE, bri.F32, bri.F32, 80, 1, 1, 1),
    "recompute_f64": (bri.RECOMPUTE, bri.F64, bri.F64, 80, 1, 1, 1),
}

# production operator (Sec. 5): name -> (w_prec, s_prec, transporter form, clover, nrhs)
PROD = {
    "prod2c_f32": (bri.F32, bri.F32, bri.W_SU3_2ROW, True, 1),
    "prod3c_f32": (bri.F32, bri.F32, bri.W_SU3, True, 1),
    "prod2_f32": (bri.F32, bri.F32, bri.W_SU3_2ROW, False, 1),
    "prod2c_f16": (bri.F16, bri.F32, bri.W_SU3_2ROW, True, 1),
    "prod2c_f64": (bri.F64, bri.F64, bri.W_SU3_2ROW, True, 1),
    "prod2c12_f32": (bri.F32, bri.F32, bri.W_SU3_2ROW, True, 12),
    "prod2c12_f16": (bri.F16, bri.F32, bri.W_SU3_2ROW, True, 12),
}


def _time(fn, reps):
    fn()
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        fn()
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / reps


def run(dims, names, reps=3, mass=0.1):
    V = bri.volume(dims)
    Ud = synth.gauge_links_device(dims, 0.3, 4001)
    U64 = bri.bri_pack_links(dims, Ud, bri.F64)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(4002)
    shp = (1,) + synth.lattice_shape(dims) + (4, 3)
    psi = torch.complex(torch.randn(shp, generator=gen, dtype=torch.float64, device="cuda"),
                        torch.randn(shp, generator=gen, dtype=torch.float64, device="cuda"))
    out = []
    for name in names:
        if name == "stream":
            big = torch.ones(1 << 30, dtype=torch.float64, device="cuda")       # 8 GiB
            ms = _time(lambda: big.sum(), reps)
            out.append({"variant": "stream_read_8GiB", "ms": ms, "GBs": big.numel() * 8 / ms / 1e6})
            del big
            a = torch.empty(1 << 31, dtype=torch.uint8, device="cuda")
            b = torch.empty_like(a)
            ms = _time(lambda: b.copy_(a), reps)
            out.append({"variant": "copy_2GiB", "ms": ms, "GBs": 2 * a.numel() / ms / 1e6})
            del a, b
            continue
        if name == "build_w80_f32":
            W = bri.bri_build_transporters(dims, U64, bri.F32, 80)
            ms = _time(lambda: bri.bri_build_transporters(dims, U64, bri.F32, 80, out=W), reps)
            out.append({"variant": name, "ms": ms, "alg_GBs": V * (576 + 5760) / ms / 1e6,
                        "fp64_TFs": V * 104 * 216 / ms / 1e9})
            del W
            torch.cuda.empty_cache()
            continue
        if name == "grad_w40":
            W40 = bri.bri_build_transporters(dims, U64, bri.F64, 40)
            chi = bri.bri_pack_spinor(dims, psi, bri.F64)
            x = bri.bri_pack_spinor(dims, psi.conj(), bri.F64)
            ms = _time(lambda: bri.bri_grad_links(dims, U64, chi, x, W40=W40), reps)
            out.append({"variant": name, "ms": ms, "alg_GBs": V * (576 + 5760 + 384 + 576) / ms / 1e6})
            del W40, chi, x
            torch.cuda.empty_cache()
            continue
        if name == "overlap_sign_24":
            out.append(_run_overlap(reps))
            torch.cuda.empty_cache()
            continue
        if name in ("wilson_f32", "wilson_f64"):
            wp = bri.F32 if name == "wilson_f32" else bri.F64
            Uw = bri.bri_pack_links(dims, Ud, wp)
            x = bri.bri_pack_spinor(dims, psi, wp)
            y = torch.empty_like(x)
            ms = _time(lambda: bri.bri_apply_wilson(dims, Uw, x, mass, out=y), reps)
            out.append({"variant": name, "ms": ms, "alg_GBs": V * 60 * CB[wp] / ms / 1e6})
            del Uw, x, y
            torch.cuda.empty_cache()
            continue
        if name == "mfma12_w80_f16":
            # the matrix-core apply of the 12 point sources (site-major FP16
            # store from the FP32 80-offset store, site-major FP32 spinors)
            W = bri.bri_build_transporters(dims, U64, bri.F32, 80)
            Wm = bri.bri_pack_w_mfma(dims, W)
            del W
            src = torch.from_numpy(synth.point_sources(dims)).to("cuda")
            x = bri.bri_pack_spinor(dims, src, bri.F32)
            del src
            x, b2 = bri.bri_spinor_to_sites(dims, x, bound2=True)
            y = torch.empty_like(x)
            ms = _time(lambda: bri.bri_apply_mfma(dims, Wm, x, mass, bound2=b2, out=y), reps)
            out.append({"variant": name, "ms": ms, "alg_GBs": V * (80 * 9 * 4 + 2 * 12 * 12 * 8) / ms / 1e6,
                        "mfma_issued_TFs": V * 20 * 6 * 16 * 16 * 32 * 2 / ms / 1e9})
            del Wm, x, y, b2
            torch.cuda.empty_cache()
            continue
        if name in PROD:
            out.append(_run_prod(dims, name, Ud, U64, psi, reps, mass))
            torch.cuda.empty_cache()
            continue
        variant, wp, sp, noff, nrhs, kernel, rblk = VARIANTS[name]
        if nrhs == 12:
            src = torch.from_numpy(synth.point_sources(dims)).to("cuda")
            x = bri.bri_pack_spinor(dims, src, sp)
            del src
        else:
            x = bri.bri_pack_spinor(dims, psi, sp)
        if variant == bri.STORED:
            Wv = bri.bri_build_transporters(dims, U64, wp, noff)
            byts = V * (noff * 9 * CB[wp] + nrhs * 2 * 12 * CB[sp])
        else:
            Wv = bri.bri_pack_links(dims, Ud, wp)
            byts = V * (36 * CB[wp] + nrhs * 2 * 12 * CB[sp])
        bri.bri_set_apply_config(dims, wp, sp, noff, nrhs, kernel, rblk)
        y = torch.empty_like(x)
        fn = bri.bri_apply_dag if name.endswith("_dag") else bri.bri_apply
        ms = _time(lambda: fn(dims, Wv, x, mass, variant=variant, out=y), reps)
        bri.bri_set_apply_config(dims, wp, sp, noff, nrhs, -1, 0)
        out.append({"variant": name, "ms": ms, "alg_GBs": byts / ms / 1e6,
                    "nominal_TFs": 35376 * V * nrhs / ms / 1e9})
        del Wv, x, y
        torch.cuda.empty_cache()
    return out


def _run_overlap(reps):
    """sign(gamma5 D(-1)) at 24^3 x 48 (links eps 0.4, seed 3001) for the
    smeared, projected kernel, degree for 1e-10 from 300 Lanczos steps."""
    dims = (24, 24, 24, 48)
    Ud = synth.gauge_links_device(dims, 0.4, 3001)
    Us = bri.bri_ape_smear(dims, bri.bri_pack_links(dims, Ud, bri.F64), 0.72)
    del Ud
    op = bri.Operator(bri.bri_build_transporters_ex(dims, Us, bri.F64, 80, bri.W_SU3_2ROW), bri.W_SU3_2ROW)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(3003)
    shp = (1,) + synth.lattice_shape(dims) + (4, 3)
    v0 = bri.bri_pack_spinor(dims, torch.complex(torch.randn(shp, generator=gen, dtype=torch.float64, device="cuda"),
                                                 torch.randn(shp, generator=gen, dtype=torch.float64, device="cuda")),
                             bri.F64)
    a, b, _ = bri.bri_lanczos(dims, op, -1.0, 300, v0)
    r = bri.bri_ritz_values(a, b)
    lo, hi = 0.9 * r[0], 1.05 * r[-1]
    deg = bri.sign_degree(lo, hi, 1e-10)
    y = torch.empty_like(v0)
    ms = _time(lambda: bri.bri_sign_h(dims, op, -1.0, v0, lo, hi, deg, out=y, with_error=False), reps)
    return {"variant": "overlap_sign_24", "ms": ms, "degree": deg, "D_applies": 2 * deg + 3,
            "ms_per_D_apply": ms / (2 * deg + 3), "ritz": [float(r[0]), float(r[-1])]}


def _run_prod(dims, name, Ud, U64, psi, reps, mass):
    wp, sp, form, clover, nrhs = PROD[name]
    V = bri.volume(dims)
    Us = bri.bri_ape_smear(dims, U64, 0.72)
    W = bri.bri_build_transporters_ex(dims, Us, wp, 80, form)
    C = bri.bri_build_clover(dims, Us, 1.0, sp) if clover else None
    op = bri.Operator(W, form, C)
    if nrhs == 12:
        src = torch.from_numpy(synth.point_sources(dims)).to("cuda")
        x = bri.bri_pack_spinor(dims, src, sp)
        del src
    else:
        x = bri.bri_pack_spinor(dims, psi, sp)
    y = torch.empty_like(x)
    ms = _time(lambda: bri.bri_apply_op(dims, op, x, mass, out=y), reps)
    rows = 6 if form == bri.W_SU3_2ROW else 9
    byts = V * (80 * rows * CB[wp] + nrhs * 2 * 12 * CB[sp] + (36 * CB[sp] if clover else 0))
    return {"variant": name, "ms": ms, "alg_GBs": byts / ms / 1e6, "alg_bytes_per_site": byts // V}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--dims", type=int, nargs=4, default=[32, 32, 32, 64])
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--variants", nargs="+", default=["tile_w80_f32"])
    a = ap.parse_args()
    for r in run(tuple(a.dims), a.variants, a.reps):
        print(json.dumps(r), flush=True)


if __name__ == "__main__":
    main()
