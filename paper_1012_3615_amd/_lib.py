"""ctypes prototypes of the C ABI in include/bri.h (libbri.so, built in-tree)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbri.so")


class bri_dims(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32 * 4)]


class bri_solve_params(ctypes.Structure):
    _fields_ = [
        ("tol", ctypes.c_double),
        ("inner_tol", ctypes.c_double),
        ("max_iter", ctypes.c_int32),
        ("max_outer", ctypes.c_int32),
        ("n_offsets", ctypes.c_int32),
        ("inner_prec", ctypes.c_int32),
        ("check_every", ctypes.c_int32),
        ("use_initial_guess", ctypes.c_int32),
        ("dagger", ctypes.c_int32),
        ("inner_mfma", ctypes.c_int32),
    ]


BRI_MAX_RHS = 64


class bri_solve_stats(ctypes.Structure):
    _fields_ = [
        ("iterations", ctypes.c_int32),
        ("outer", ctypes.c_int32),
        ("applies", ctypes.c_int32),
        ("converged", ctypes.c_int32),
        ("true_residual", ctypes.c_double * BRI_MAX_RHS),
    ]


# BRI_ABI_VERSION of include/bri.h that the structures below mirror
ABI_VERSION = 6


class bri_operator(ctypes.Structure):
    _fields_ = [
        ("W", ctypes.c_void_p),
        ("w_prec", ctypes.c_int32),
        ("n_offsets", ctypes.c_int32),
        ("w_form", ctypes.c_int32),
        ("clover", ctypes.c_void_p),
        ("coef", ctypes.c_void_p),
    ]


_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_sz = ctypes.c_size_t
_dbl = ctypes.c_double
_D = bri_dims

# name -> (restype, argtypes)
PROTOTYPES = {
    "bri_last_error": (ctypes.c_char_p, []),
    "bri_abi_version": (_i32, []),
    "bri_spinor_bytes": (_sz, [_D, _i32, _i32]),
    "bri_links_bytes": (_sz, [_D, _i32]),
    "bri_transporter_bytes": (_sz, [_D, _i32, _i32]),
    "bri_pack_links": (_i32, [_D, _vp, _vp, _i32, _vp]),
    "bri_pack_spinor": (_i32, [_D, _i32, _vp, _vp, _i32, _vp]),
    "bri_unpack_spinor": (_i32, [_D, _i32, _vp, _i32, _vp, _vp]),
    "bri_unpack_links": (_i32, [_D, _vp, _i32, _vp, _vp]),
    "bri_build_workspace_bytes": (_sz, [_D, _i32, _i32]),
    "bri_build_transporters": (_i32, [_D, _vp, _vp, _i32, _i32, _vp, _sz, _vp]),
    "bri_apply": (_i32, [_D, _i32, _vp, _i32, _i32, _i32, _dbl, _vp, _vp, _i32, _vp]),
    "bri_apply_dag": (_i32, [_D, _i32, _vp, _i32, _i32, _i32, _dbl, _vp, _vp, _i32, _vp]),
    "bri_apply_wilson": (_i32, [_D, _vp, _i32, _dbl, _vp, _vp, _i32, _i32, _vp]),
    "bri_pack_w_mfma": (_i32, [_D, _vp, _i32, _i32, _vp, _vp]),
    "bri_spinor_bound2": (_i32, [_D, _i32, _vp, _vp, _vp]),
    "bri_spinor_to_sites": (_i32, [_D, _i32, _vp, _vp, _vp, _vp]),
    "bri_spinor_from_sites": (_i32, [_D, _i32, _vp, _vp, _vp]),
    "bri_apply_mfma": (_i32, [_D, _vp, _dbl, _vp, _vp, _i32, _i32, _vp, _vp, _vp]),
    "bri_set_apply_config": (_i32, [_D, _i32, _i32, _i32, _i32, _i32, _i32]),
    "bri_get_apply_config": (_i32, [_D, _i32, _i32, _i32, _i32, ctypes.POINTER(_i32), ctypes.POINTER(_i32)]),
    "bri_clear_apply_configs": (None, []),
    "bri_solve_workspace_bytes": (_sz, [_D, ctypes.POINTER(bri_solve_params), _i32]),
    "bri_solve_cgne": (_i32, [_D, ctypes.POINTER(bri_solve_params), _vp, _vp, _dbl, _vp, _vp,
                              _i32, _vp, _sz, ctypes.POINTER(bri_solve_stats), _vp]),
    "bri_solve_cgne_noalloc": (_i32, [_D, ctypes.POINTER(bri_solve_params), _vp, _vp, _dbl, _vp, _vp,
                                      _i32, ctypes.POINTER(bri_solve_stats), _vp]),
    "bri_grad_workspace_bytes": (_sz, [_D]),
    "bri_grad_links": (_i32, [_D, _vp, _vp, _vp, _i32, _dbl, _vp, _vp, _vp, _sz, _vp]),
    "bri_grad_workspace_bytes_w": (_sz, [_D]),
    "bri_grad_links_w": (_i32, [_D, _vp, _vp, _vp, _vp, _i32, _dbl, _vp, _vp, _vp, _sz, _vp]),
    "bri_project_su3": (_i32, [ctypes.c_int64, _vp, _vp, _vp]),
    "bri_ape_smear": (_i32, [_D, _vp, _vp, _dbl, _vp]),
    "bri_transporter_bytes_ex": (_sz, [_D, _i32, _i32, _i32]),
    "bri_build_workspace_bytes_ex": (_sz, [_D, _i32, _i32, _i32]),
    "bri_build_transporters_ex": (_i32, [_D, _vp, _vp, _i32, _i32, _i32, _vp, _sz, _vp]),
    "bri_clover_bytes": (_sz, [_D, _i32]),
    "bri_build_clover": (_i32, [_D, _vp, _dbl, _vp, _i32, _vp]),
    "bri_apply_op": (_i32, [_D, ctypes.POINTER(bri_operator), _i32, _dbl, _vp, _vp, _i32, _i32, _vp]),
    "bri_solve_cgne_op": (_i32, [_D, ctypes.POINTER(bri_solve_params), ctypes.POINTER(bri_operator),
                                 ctypes.POINTER(bri_operator), _dbl, _vp, _vp, _i32, _vp, _sz,
                                 ctypes.POINTER(bri_solve_stats), _vp]),
    "bri_lanczos_workspace_bytes": (_sz, [_D, _i32]),
    "bri_lanczos": (_i32, [_D, ctypes.POINTER(bri_operator), _dbl, _i32, _vp, _vp, _vp, _vp,
                           ctypes.POINTER(_i32), _vp, _sz, _vp]),
    "bri_ritz_values": (_i32, [_i32, _vp, _vp, _i32, _vp, ctypes.POINTER(_i32)]),
    "bri_lowmodes_workspace_bytes": (_sz, [_D, _i32, _i32]),
    "bri_overlap_lowmodes": (_i32, [_D, ctypes.POINTER(bri_operator), _dbl, _i32, _vp, _i32, _vp, _vp, _vp, _vp,
                                    _vp, _sz, _vp]),
    "bri_sign_workspace_bytes": (_sz, [_D, _i32]),
    "bri_sign_approx_error": (_i32, [_dbl, _dbl, _i32, ctypes.POINTER(_dbl)]),
    "bri_sign_h": (_i32, [_D, ctypes.POINTER(bri_operator), _dbl, _dbl, _dbl, _i32, _i32, _vp, _vp, _vp, _vp,
                          _i32, ctypes.POINTER(_dbl), _vp, _sz, _vp]),
    "bri_overlap_apply": (_i32, [_D, ctypes.POINTER(bri_operator), _dbl, _dbl, _dbl, _dbl, _i32, _i32, _vp,
                                 _vp, _vp, _vp, _i32, ctypes.POINTER(_dbl), _vp, _sz, _vp]),
}


def load(path=LIB_PATH):
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is missing: build the HIP library first "
            "(python -m paper_1012_3615_amd.build or __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    for name, (res, args) in PROTOTYPES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if lib.bri_abi_version() != ABI_VERSION:
        raise ImportError(f"{path} implements ABI revision {lib.bri_abi_version()}, this binding "
                          f"revision {ABI_VERSION}: rebuild the library")
    return lib
