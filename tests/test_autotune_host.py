"""Host-side state of the autotuner (no GPU needed): an installed choice is
per precision pair and reset() restores the built-in selection."""
import pytest


def test_reset_restores_builtin_selection():
    import paper_1012_3615_amd as bri
    from paper_1012_3615_amd import autotune
    assert (bri.bri_get_apply_kernel(bri.F32, bri.F32), bri.bri_get_rhs_block(bri.F32, bri.F32)) == (1, 2)
    try:
        autotune._install(bri.F32, bri.F32, 8, 1)
        assert (bri.bri_get_apply_kernel(bri.F32, bri.F32), bri.bri_get_rhs_block(bri.F32, bri.F32)) == (8, 1)
        # other precision pairs are untouched
        assert bri.bri_get_apply_kernel(bri.F64, bri.F64) == 1
        autotune.reset(bri.F32, bri.F32)
        assert (bri.bri_get_apply_kernel(bri.F32, bri.F32), bri.bri_get_rhs_block(bri.F32, bri.F32)) == (1, 2)
    finally:
        autotune.reset(bri.F32, bri.F32)


def test_invalid_choices_are_rejected():
    import paper_1012_3615_amd as bri
    with pytest.raises(Exception):
        bri.bri_set_apply_kernel(bri.F32, bri.F32, 15)
    with pytest.raises(Exception):
        bri.bri_set_rhs_block(bri.F32, bri.F32, 5)
    assert bri.bri_get_apply_kernel(bri.F32, bri.F32) == 1
