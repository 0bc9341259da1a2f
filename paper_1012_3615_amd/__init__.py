"""MI355X (gfx950) Brillouin Dirac operator: HIP kernels behind a C ABI.

Importing the package loads the in-tree HIP library ``libbri.so``; there is
no fallback implementation, so the import fails loudly when the library has
not been built.
"""
from .api import (  # noqa: F401
    F64, F32, F16, STORED, RECOMPUTE, BriError, volume,
    spinor_empty, links_empty, transporters_empty,
    bri_pack_links, bri_pack_spinor, bri_unpack_spinor, bri_unpack_links,
    bri_build_transporters, bri_apply, bri_apply_dag, bri_apply_wilson,
    bri_pack_w_mfma, bri_spinor_bound2, bri_apply_mfma, bri_spinor_to_sites, bri_spinor_from_sites,
    bri_set_apply_config, bri_get_apply_config, bri_clear_apply_configs,
    solve_params, bri_solve_cgne, bri_solve_cgne_noalloc, bri_grad_links,
    W_AVERAGE, W_SU3, W_SU3_2ROW, Operator, bri_project_su3, bri_ape_smear, bri_build_transporters_ex,
    bri_build_clover, bri_apply_op, bri_solve_cgne_op,
    bri_lanczos, bri_ritz_values, bri_sign_h, bri_overlap_apply, bri_sign_approx_error, sign_degree,
    bri_overlap_lowmodes, TABLE_WILSON, TABLE_HYPERCUBE, TABLE_BRILLOUIN,
)
