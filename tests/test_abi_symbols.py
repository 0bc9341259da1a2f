"""Host-side checks of the C ABI library (no GPU needed): it loads and exports
every function declared in include/bri.h, and the pure size queries agree
with the documented layouts."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bri.h")
LIB = os.path.join(ROOT, "paper_1012_3615_amd", "libbri.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(bri_[a-z0-9_]+)\s*\(", src)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libbri.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["bri_build_transporters", "bri_apply", "bri_apply_dag", "bri_solve_cgne",
                     "bri_grad_links", "bri_pack_links", "bri_pack_spinor", "bri_unpack_spinor"]:
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_python_prototypes_cover_header():
    from paper_1012_3615_amd import _lib as plib
    assert set(declared_functions()) <= set(plib.PROTOTYPES)


def test_size_queries(lib):
    from paper_1012_3615_amd import _lib as plib
    for name, (res, args) in plib.PROTOTYPES.items():
        getattr(lib, name).restype = res
        getattr(lib, name).argtypes = args
    d = plib.bri_dims()
    for i, v in enumerate((32, 32, 32, 64)):
        d.L[i] = v
    V = 32 ** 3 * 64
    assert lib.bri_spinor_bytes(d, 1, 1) == V * 12 * 8
    assert lib.bri_spinor_bytes(d, 0, 12) == V * 12 * 16 * 12
    assert lib.bri_links_bytes(d, 0) == V * 36 * 16
    assert lib.bri_transporter_bytes(d, 1, 80) == V * 80 * 9 * 8
    assert lib.bri_transporter_bytes(d, 2, 40) == V * 40 * 9 * 4
    assert lib.bri_transporter_bytes(d, 1, 39) == 0
    assert lib.bri_build_workspace_bytes(d, 0, 40) == 0
    assert lib.bri_build_workspace_bytes(d, 1, 80) == 0  # the fused build needs no stage
    assert lib.bri_abi_version() == plib.ABI_VERSION == 6
    # production-operator forms: two-row SU(3) store and the clover term
    assert lib.bri_transporter_bytes_ex(d, 1, 80, 0) == V * 80 * 9 * 8
    assert lib.bri_transporter_bytes_ex(d, 1, 80, 1) == V * 80 * 9 * 8
    assert lib.bri_transporter_bytes_ex(d, 1, 80, 2) == V * 80 * 6 * 8
    assert lib.bri_transporter_bytes_ex(d, 1, 80, 3) == 0
    assert lib.bri_build_workspace_bytes_ex(d, 0, 40, 1) == 0
    assert lib.bri_build_workspace_bytes_ex(d, 0, 40, 2) == V * 40 * 9 * 16
    assert lib.bri_clover_bytes(d, 1) == V * 36 * 8
    assert lib.bri_clover_bytes(d, 0) == V * 36 * 16
    d.L[3] = 1
    assert lib.bri_spinor_bytes(d, 1, 1) == 0


def test_argument_errors_without_device(lib):
    """Argument validation happens before any device work: null pointers and
    bad extents are rejected with BRI_E_ARG and a message."""
    from paper_1012_3615_amd import _lib as plib
    for name, (res, args) in plib.PROTOTYPES.items():
        getattr(lib, name).restype = res
        getattr(lib, name).argtypes = args
    d = plib.bri_dims()
    for i in range(4):
        d.L[i] = 4
    st = lib.bri_apply(d, 0, None, 1, 80, 1, 0.1, None, None, 1, None)
    assert st == -1
    assert b"pointer" in lib.bri_last_error()
    assert lib.bri_project_su3(-1, None, None, None) == -1
    assert lib.bri_project_su3(0, None, None, None) == 0
    assert lib.bri_apply_op(d, None, 1, 0.1, None, None, 1, 0, None) == -1
    assert b"operator" in lib.bri_last_error()
    op = plib.bri_operator()
    op.w_form = 7
    assert lib.bri_apply_op(d, ctypes.byref(op), 1, 0.1, None, None, 1, 0, None) == -1
    assert b"form" in lib.bri_last_error()
    assert lib.bri_apply_wilson(d, None, 1, 0.1, None, None, 1, 0, None) == -1
    assert b"pointer" in lib.bri_last_error()
    assert lib.bri_apply_wilson(d, None, 2, 0.1, None, None, 1, 0, None) == -2
    assert lib.bri_apply_wilson(d, None, 1, 0.1, None, None, 1, 2, None) == -1
    assert lib.bri_build_transporters_ex(d, None, None, 1, 80, 2, None, 0, None) == -1
    # the matrix-core apply: argument checks come before any device work
    assert lib.bri_apply_mfma(d, None, 0.1, None, None, 12, 0, None, None, None) == -1
    assert b"pointer" in lib.bri_last_error()
    assert lib.bri_apply_mfma(d, None, 0.1, None, None, 0, 0, None, None, None) == -1
    assert b"nrhs" in lib.bri_last_error()
    assert lib.bri_apply_mfma(d, None, 0.1, None, None, 12, 3, None, None, None) == -1
    assert b"dagger" in lib.bri_last_error()
    assert lib.bri_pack_w_mfma(d, None, 1, 39, None, None) == -1
    assert b"n_offsets" in lib.bri_last_error()
    assert lib.bri_pack_w_mfma(d, None, 5, 80, None, None) == -1
    assert lib.bri_spinor_bound2(d, 0, None, None, None) == -1
    assert lib.bri_ape_smear(d, None, None, 0.72, None) == -1
    assert lib.bri_build_clover(d, None, 1.0, None, 1, None) == -1
    d.L[0] = 1
    st = lib.bri_build_transporters(d, None, None, 0, 80, None, 0, None)
    assert st == -1
