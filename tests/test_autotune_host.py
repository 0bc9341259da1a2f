"""Host-side state of the launch configurations (no GPU needed): an installed
choice belongs to one shape (extents, precisions, offsets, right-hand sides)
and the built-in selection resolves to the tiles the benchmark times."""
import pytest

BENCH = (32, 32, 32, 64)


def test_builtin_selection_resolves_to_the_benchmarked_tiles():
    import paper_1012_3615_amd as bri
    bri.bri_clear_apply_configs()
    # one right-hand side, FP32 or FP64, 80 offsets: the 32x16 tile (code 13)
    assert bri.bri_get_apply_config(BENCH, bri.F32, bri.F32, 80, 1) == (13, 1)
    assert bri.bri_get_apply_config(BENCH, bri.F64, bri.F64, 80, 1) == (13, 1)
    # FP16 transporters and the 40-offset store: 32x8 with prefetch (code 8)
    assert bri.bri_get_apply_config(BENCH, bri.F16, bri.F32, 80, 1) == (8, 1)
    assert bri.bri_get_apply_config(BENCH, bri.F32, bri.F32, 40, 1) == (8, 1)
    # twelve right-hand sides: 32x8 with two per thread
    assert bri.bri_get_apply_config(BENCH, bri.F32, bri.F32, 80, 12) == (8, 2)
    # widths that follow Lx
    assert bri.bri_get_apply_config((24, 24, 24, 48), bri.F32, bri.F32, 80, 1) == (11, 1)
    assert bri.bri_get_apply_config((48, 8, 2, 2), bri.F32, bri.F32, 80, 1) == (12, 1)
    assert bri.bri_get_apply_config((16, 16, 16, 32), bri.F32, bri.F32, 80, 1) == (14, 1)
    assert bri.bri_get_apply_config((16, 16, 16, 32), bri.F64, bri.F64, 80, 1) == (7, 1)
    assert bri.bri_get_apply_config((8, 8, 8, 8), bri.F64, bri.F64, 80, 12) == (10, 2)


def test_installed_choice_is_per_shape():
    import paper_1012_3615_amd as bri
    from paper_1012_3615_amd import autotune
    bri.bri_clear_apply_configs()
    try:
        autotune.install(BENCH, bri.F32, bri.F32, 80, 12, 0, 6)
        assert bri.bri_get_apply_config(BENCH, bri.F32, bri.F32, 80, 12) == (0, 6)
        # every other shape keeps the built-in selection
        assert bri.bri_get_apply_config(BENCH, bri.F32, bri.F32, 80, 1) == (13, 1)
        assert bri.bri_get_apply_config(BENCH, bri.F32, bri.F32, 80, 11) == (8, 2)
        assert bri.bri_get_apply_config(BENCH, bri.F32, bri.F32, 40, 12) == (8, 2)
        assert bri.bri_get_apply_config(BENCH, bri.F64, bri.F64, 80, 12) == (8, 2)
        assert bri.bri_get_apply_config((32, 32, 32, 32), bri.F32, bri.F32, 80, 12) == (8, 2)
        # re-installing replaces; the blocking is clamped to what a tile holds
        autotune.install(BENCH, bri.F32, bri.F32, 80, 12, 8, 4)
        assert bri.bri_get_apply_config(BENCH, bri.F32, bri.F32, 80, 12) == (8, 2)
        autotune.reset(BENCH, bri.F32, bri.F32, 80, 12)
        assert bri.bri_get_apply_config(BENCH, bri.F32, bri.F32, 80, 12) == (8, 2)
        # removing an absent entry is harmless
        autotune.reset(BENCH, bri.F32, bri.F32, 80, 12)
    finally:
        bri.bri_clear_apply_configs()


def test_table_capacity_and_invalid_choices():
    import paper_1012_3615_amd as bri
    bri.bri_clear_apply_configs()
    try:
        with pytest.raises(bri.BriError):
            bri.bri_set_apply_config(BENCH, bri.F32, bri.F32, 80, 1, 15, 1)
        with pytest.raises(bri.BriError):
            bri.bri_set_apply_config(BENCH, bri.F32, bri.F32, 80, 2, 2, 5)
        with pytest.raises(bri.BriError):
            bri.bri_set_apply_config(BENCH, bri.F32, bri.F32, 60, 2, 2, 2)
        with pytest.raises(bri.BriError):
            bri.bri_set_apply_config((1, 4, 4, 4), bri.F32, bri.F32, 80, 2, 2, 2)
        assert bri.bri_get_apply_config(BENCH, bri.F32, bri.F32, 80, 1) == (13, 1)
        for n in range(1, 257):
            bri.bri_set_apply_config(BENCH, bri.F32, bri.F32, 80, n, 0, 1)
        with pytest.raises(bri.BriError):
            bri.bri_set_apply_config(BENCH, bri.F32, bri.F32, 80, 257, 0, 1)
        # replacing an existing entry still works at capacity
        bri.bri_set_apply_config(BENCH, bri.F32, bri.F32, 80, 5, 2, 4)
        assert bri.bri_get_apply_config(BENCH, bri.F32, bri.F32, 80, 5) == (2, 4)
    finally:
        bri.bri_clear_apply_configs()
    assert bri.bri_get_apply_config(BENCH, bri.F32, bri.F32, 80, 5) == (8, 2)
