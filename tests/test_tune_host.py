"""Host side of the launch-shape table: storing, looking up, validating and
forgetting shapes, and argument checks of the tuner (no device needed)."""

import ctypes

import pytest

import paper_2007_06483_amd as mtb


@pytest.fixture(autouse=True)
def clean_table():
    mtb.mtb_tune_reset()
    yield
    mtb.mtb_tune_reset()


def test_set_lookup_and_reset():
    key = (7, 6000, 4000, 18000, 7)
    assert mtb.mtb_tuned_shape(*key) is None
    mtb.mtb_set_shape(*key, {"pyramid_slots_pct": 200, "pyramid_tile_group": 2, "bitmaps_blocks_pct": 75,
                             "bitmaps_waves": 8, "coarse_levels": 2, "small_search": 0, "level1_from_level0": 0,
                             "search_rows": [8, 0, 16], "search_lanes": [0, 16, 64]})
    got = mtb.mtb_tuned_shape(*key)
    assert got["pyramid_slots_pct"] == 200 and got["bitmaps_blocks_pct"] == 75
    assert got["pyramid_tile_group"] == 2 and got["bitmaps_waves"] == 8 and got["coarse_levels"] == 2
    assert got["small_search"] == 0 and got["level1_from_level0"] == 0
    assert got["search_rows"][:4] == [8, 0, 16, 0]
    assert got["search_lanes"][:4] == [0, 16, 64, 0]
    # The key distinguishes image count, size, levels and the row-stride class.
    assert mtb.mtb_tuned_shape(6, 6000, 4000, 18000, 7) is None
    assert mtb.mtb_tuned_shape(7, 6000, 4000, 18000, 6) is None
    assert mtb.mtb_tuned_shape(7, 6000, 4000, 18004, 7) is None       # stride class 4, not 16
    assert mtb.mtb_tuned_shape(7, 6000, 4000, 18016, 7) is not None   # same class 16
    mtb.mtb_tune_reset()
    assert mtb.mtb_tuned_shape(*key) is None


@pytest.mark.parametrize("bad", [
    {"pyramid_slots_pct": 24}, {"pyramid_slots_pct": 401}, {"bitmaps_blocks_pct": 24},
    {"bitmaps_blocks_pct": 101}, {"search_rows": [2]}, {"search_rows": [6]}, {"search_rows": [68]},
    {"search_rows": [0, -4]}, {"pyramid_tile_group": 3}, {"pyramid_tile_group": 0}, {"bitmaps_waves": 1},
    {"bitmaps_waves": 16}, {"coarse_levels": -2}, {"coarse_levels": 6}, {"small_search": 2},
    {"small_search": -2}, {"level1_from_level0": 2}, {"level1_from_level0": -2}, {"search_lanes": [4]},
    {"search_lanes": [0, 128]}, {"search_lanes": [24]},
])
def test_out_of_range_shapes_are_refused(bad):
    shape = {"pyramid_slots_pct": 100, "bitmaps_blocks_pct": 100, "search_rows": []}
    shape.update(bad)
    with pytest.raises(RuntimeError):
        mtb.mtb_set_shape(7, 640, 480, 1920, 5, shape)
    assert mtb.mtb_tuned_shape(7, 640, 480, 1920, 5) is None


def test_a_shape_serves_its_size_bucket():
    # 6000x4000 and 6100x3950 share the half-octave bucket round(2 log2(w h)) = 49
    # (same images, levels and stride class); 3000x2000 (bucket 45) does not.
    mtb.mtb_set_shape(7, 6000, 4000, 18000, 7, {"pyramid_slots_pct": 150, "search_rows": [12]})
    near = mtb.mtb_tuned_shape(7, 6100, 3950, 18304, 7)
    assert near is not None and near["pyramid_slots_pct"] == 150 and near["search_rows"][0] == 12
    assert mtb.mtb_tuned_shape(7, 3000, 2000, 9008, 7) is None
    assert mtb.mtb_tuned_shape(6, 6100, 3950, 18304, 7) is None    # image count differs
    assert mtb.mtb_tuned_shape(7, 6100, 3950, 18302, 7) is None    # stride class 1
    # A size's own shape wins over its bucket's.
    mtb.mtb_set_shape(7, 6100, 3950, 18304, 7, {"pyramid_slots_pct": 50})
    assert mtb.mtb_tuned_shape(7, 6100, 3950, 18304, 7)["pyramid_slots_pct"] == 50


def test_save_and_load_need_a_device():
    # The file records the device architecture and HIP version, so without a
    # device neither call can run; bad arguments are refused first.
    L = mtb.lib()
    n = ctypes.c_int32(-1)
    assert L.mtb_tune_save(None) == 1
    assert L.mtb_tune_load(None, ctypes.byref(n)) == 1
    assert L.mtb_tune_load(b"/nonexistent", None) == 1


def test_invalid_keys_are_refused():
    ok = {"pyramid_slots_pct": 100, "bitmaps_blocks_pct": 100}
    for key in [(0, 640, 480, 1920, 5), (33, 640, 480, 1920, 5), (7, 640, 480, 1919, 5),
                (7, 640, 480, 1920, 0), (7, 640, 480, 1920, 20), (7, 0, 480, 1920, 5)]:
        with pytest.raises(RuntimeError):
            mtb.mtb_set_shape(*key, ok)


def test_tuner_argument_checks():
    L = mtb.lib()
    FAKE, NULL = ctypes.c_void_p(0x1000), None
    ptrs = (ctypes.c_void_p * 2)(0x1000, 0x2000)
    out = mtb._LaunchShape()
    ws = mtb.mtb_stack_workspace_bytes(2, 64, 48, 3)
    args = [ptrs, 2, 64, 48, 192, 3, 4, -1, FAKE, ws, FAKE, FAKE, NULL, ctypes.byref(out)]
    for i, v in ((0, NULL), (1, 0), (2, 0), (4, 191), (5, 0), (6, 256), (7, 2), (8, NULL), (9, ws - 1),
                 (10, NULL), (11, NULL), (13, NULL)):
        bad = list(args)
        bad[i] = v
        assert L.mtb_tune_stack(*bad) in (1, 2), (i, v)   # MTB_ERR_INVALID_ARG or MTB_ERR_WORKSPACE
    assert mtb.mtb_tuned_shape(2, 64, 48, 192, 3) is None
