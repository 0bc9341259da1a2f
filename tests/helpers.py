"""Shared helpers for the GPU tests: move seeded synthetic inputs to the
device and bring results back in the oracle's canonical layout."""
import sys

import numpy as np

import synth


def log(msg):
    """Name the case before each GPU step (flushed, so a crash still shows it)."""
    print(f"[gpu-case] {msg}", file=sys.stderr, flush=True)


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    return t.detach().cpu().numpy()


def soa_to_canon(dims, soa):
    """[nrhs,12,V,2] real tensor (any float dtype) -> numpy complex128
    [nrhs, Lt, Lz, Ly, Lx, 4, 3] without using the library."""
    a = host(soa).astype(np.float64)
    c = a[..., 0] + 1j * a[..., 1]               # [nrhs, 12, V]
    nrhs = c.shape[0]
    c = np.transpose(c, (0, 2, 1))               # [nrhs, V, 12]
    return c.reshape((nrhs,) + synth.lattice_shape(dims) + (4, 3))


def transporter_plane_to_canon(dims, plane):
    """[9,V,2] -> complex (Lt,Lz,Ly,Lx,3,3)."""
    a = host(plane).astype(np.float64)
    c = a[..., 0] + 1j * a[..., 1]               # [9, V]
    return c.T.reshape(synth.lattice_shape(dims) + (3, 3))


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def offset_of_index(i):
    """Offset numbering of the library: i = (nx+1) + 3(ny+1) + 9(nz+1) + 27(nt+1)."""
    return (i % 3 - 1, (i // 3) % 3 - 1, (i // 9) % 3 - 1, i // 27 - 1)


def plane_offsets(n_offsets):
    if n_offsets == 80:
        return [offset_of_index(j if j < 40 else j + 1) for j in range(80)]
    return [offset_of_index(41 + c) for c in range(40)]
