"""Autotuner for the stored-transporter apply.

For a lattice, precision pair, transporter store and number of right-hand
sides it times every launch configuration the library offers (LDS tiles of
32x8 or 16x8 sites with 1-4 right-hand sides per thread, tiles of 16x16,
64x4, 32x16 or 16x4 sites with one, or the register-blocked gather form with
1, 2, 3, 4, 6 or 12 right-hand sides per thread) with HIP events on the
current stream, and installs the fastest through bri_set_apply_config for
exactly that shape (extents, w_prec, s_prec, n_offsets, nrhs): applies of
every other shape keep their own choice or the built-in one.

Choices are cached in a JSON file keyed by the shape, the device name and a
hash of the library file, so an entry timed against another build of the
kernels is never installed without being re-timed.
"""
from __future__ import annotations

import hashlib
import json
import os

import torch

from . import _lib, api

CACHE = os.environ.get("BRI_AUTOTUNE_CACHE",
                       os.path.join(os.path.expanduser("~"), ".cache", "bri_autotune.json"))
TILES = {2: "tile32x8", 3: "tile16x16", 4: "tile64x4", 5: "tile16x8", 6: "tile32x8pf", 7: "tile16x16pf",
         8: "tile32x8pfu", 9: "tile32x8u", 10: "tile16x8u", 11: "tile24x8pfu", 12: "tile48x4pfu",
         13: "tile32x16pfu", 14: "tile16x4pfu"}
TILE_X = {2: 32, 3: 16, 4: 64, 5: 16, 6: 32, 7: 16, 8: 32, 9: 32, 10: 16, 11: 24, 12: 48, 13: 32, 14: 16}
# right-hand sides per thread instantiated for each tile code
TILE_RBLK = {2: (1, 2, 3, 4), 3: (1,), 4: (1,), 5: (1, 2, 3, 4), 6: (1, 2), 7: (1,), 8: (1, 2),
             9: (1, 2, 3), 10: (2, 3, 4), 11: (1, 2), 12: (1, 2), 13: (1,), 14: (1,)}
RBLKS = (1, 2, 3, 4, 6, 12)

_lib_digest = None


def library_digest():
    """sha256 (first 16 hex digits) of the loaded libbri.so and its ABI revision."""
    global _lib_digest
    if _lib_digest is None:
        h = hashlib.sha256()
        with open(_lib.LIB_PATH, "rb") as f:
            for chunk in iter(lambda: f.read(1 << 22), b""):
                h.update(chunk)
        _lib_digest = f"abi{_lib.ABI_VERSION}-{h.hexdigest()[:16]}"
    return _lib_digest


def _key(dims, w_prec, s_prec, n_offsets, nrhs):
    dev = torch.cuda.get_device_name()
    return (f"{'x'.join(map(str, dims))}|w{w_prec}|s{s_prec}|o{n_offsets}|r{nrhs}|{dev}|"
            f"{library_digest()}")


def _load():
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(c):
    try:
        os.makedirs(os.path.dirname(CACHE), exist_ok=True)
        with open(CACHE, "w") as f:
            json.dump(c, f, indent=1, sort_keys=True)
    except OSError:
        pass


def candidates(dims, nrhs, s_prec=api.F32):
    out = []
    for code, name in TILES.items():
        tx = TILE_X[code]
        if tx > 2 * dims[0]:
            continue
        for r in TILE_RBLK[code]:
            if r > nrhs:
                continue
            if r > 2 and tx == 32 and s_prec == api.F64:
                continue  # the LDS of a 32x8 tile holds at most 2 FP64 spinors
            out.append((f"{name}_r{r}", code, r))
    for r in RBLKS:
        if r <= nrhs:
            out.append((f"gather_r{r}", 0, r))
    return out


def install(dims, w_prec, s_prec, n_offsets, nrhs, kernel, rblk):
    api.bri_set_apply_config(dims, w_prec, s_prec, n_offsets, nrhs, kernel, rblk)


def reset(dims, w_prec, s_prec, n_offsets, nrhs):
    """Return one shape to the built-in selection."""
    api.bri_set_apply_config(dims, w_prec, s_prec, n_offsets, nrhs, -1, 0)


def tune(dims, W, psi, mass=0.1, reps=5, use_cache=True):
    """Pick and install the fastest configuration for apply(W, psi), for this
    shape only.  Returns (name, ms, table of all timings, from_cache); with a
    cached entry nothing is timed and the table is the one stored with it."""
    w_prec, s_prec = api.prec_of(W), api.prec_of(psi)
    n_off, nrhs = W.shape[0], psi.shape[0]
    key = _key(dims, w_prec, s_prec, n_off, nrhs)
    cache = _load() if use_cache else {}
    if key in cache:
        e = cache[key]
        install(dims, w_prec, s_prec, n_off, nrhs, e["kernel"], e["rblk"])
        return e["name"], e["ms"], e.get("table", {}), True
    out = torch.empty_like(psi)
    table = {}
    best = None
    for name, kernel, rblk in candidates(dims, nrhs, s_prec):
        install(dims, w_prec, s_prec, n_off, nrhs, kernel, rblk)
        api.bri_apply(dims, W, psi, mass, out=out)
        torch.cuda.synchronize()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        for _ in range(reps):
            api.bri_apply(dims, W, psi, mass, out=out)
        e.record()
        torch.cuda.synchronize()
        ms = s.elapsed_time(e) / reps
        table[name] = ms
        if best is None or ms < best[3]:
            best = (name, kernel, rblk, ms)
    name, kernel, rblk, ms = best
    install(dims, w_prec, s_prec, n_off, nrhs, kernel, rblk)
    if use_cache:
        cache[key] = {"name": name, "kernel": kernel, "rblk": rblk, "ms": ms, "table": table}
        _store(cache)
    return name, ms, table, False
