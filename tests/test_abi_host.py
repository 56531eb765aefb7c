"""Host-side checks of the C ABI: the library loads, exports every declared
symbol, reports the documented layout, and rejects bad arguments before
enqueuing anything.  No GPU is needed (no call here reaches a kernel)."""

import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mtb.h")


@pytest.fixture(scope="module")
def mtb():
    import paper_2007_06483_amd as m

    if not os.path.exists(m.library_path()):
        from paper_2007_06483_amd import _build

        _build.build()
    m.lib()
    return m


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mtb_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for f in ("mtb_build_pyramid", "mtb_bitmaps", "mtb_align_pair", "mtb_align_stack"):
        assert f in names


def test_library_exports_every_declared_symbol(mtb):
    lib = ctypes.CDLL(mtb.library_path())
    for name in _declared():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", mtb.library_path()], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (mtb_\w+)", out))
    assert set(_declared()) <= exported


def test_status_strings(mtb):
    assert mtb.mtb_status_string(0) == "MTB_OK"
    assert mtb.mtb_status_string(2) == "MTB_ERR_WORKSPACE"
    assert mtb.mtb_status_string(99) == "MTB_ERR_UNKNOWN"


@pytest.mark.parametrize("w,h,L", [(1, 1, 1), (2, 1, 1), (6000, 4000, 12), (512, 384, 9),
                                   (46340, 46340, 16), (1 << 30, 1, 1), (3, 1 << 20, 2)])
def test_max_levels(mtb, w, h, L):
    assert mtb.mtb_max_levels(w, h) == L


def test_max_levels_rejects_empty(mtb):
    assert mtb.mtb_max_levels(0, 5) == 0
    assert mtb.mtb_max_levels(5, -1) == 0


@pytest.mark.parametrize("w,h,L", [(6000, 4000, 7), (641, 479, 7), (1, 1, 1), (65, 3, 2)])
def test_layout_is_consistent(mtb, w, h, L):
    lay = mtb.mtb_get_layout(w, h, L)
    assert lay.levels == L
    end = 0
    for l in range(L):
        assert lay.level_width[l] == w >> l and lay.level_height[l] == h >> l
        assert lay.words_per_row[l] == 2 * -(-(w >> l) // 128)
        assert lay.gray_pitch[l] == 64 * lay.words_per_row[l]
        assert lay.gray_pitch[l] % 128 == 0
        assert lay.gray_offset[l] % 256 == 0 and lay.gray_offset[l] >= end
        end = lay.gray_offset[l] + lay.gray_pitch[l] * lay.level_height[l]
    assert lay.hist_offset >= end and lay.hist_offset % 256 == 0
    assert lay.pyramid_bytes >= lay.hist_offset + 1024 * L
    # After the histograms: the pyramid pass's merge scratch, one uint32[7][256]
    # copy per XCD (8) and the tickets; the buffer ends on a 256-byte boundary.
    assert lay.pyramid_bytes >= lay.hist_offset + 1024 * L + 8 * 7 * 1024
    assert lay.pyramid_bytes % 256 == 0
    assert lay.pyramid_bytes == mtb.mtb_pyramid_bytes(w, h, L)
    end = 0
    for l in range(L):
        plane = 8 * lay.words_per_row[l] * lay.level_height[l]
        for off in (lay.tb_offset[l], lay.eb_offset[l]):
            assert off % 256 == 0 and off >= end
            end = off + plane
    assert lay.median_offset >= end
    assert lay.bitmaps_bytes >= lay.median_offset + 4 * L
    assert lay.bitmaps_bytes == mtb.mtb_bitmaps_bytes(w, h, L)


def test_workspace_sizes(mtb):
    P, B = mtb.mtb_pyramid_bytes(6000, 4000, 7), mtb.mtb_bitmaps_bytes(6000, 4000, 7)
    ws = mtb.mtb_stack_workspace_bytes(7, 6000, 4000, 7)
    # Room for every image's pyramid and bitmaps, plus search state for the pairs.
    assert ws > 7 * (P + B)
    assert mtb.mtb_pair_workspace_bytes(7) >= 4 * 7 * 9  # at least nine counters per level
    assert mtb.mtb_stack_workspace_bytes(0, 10, 10, 1) == 0
    assert mtb.mtb_stack_workspace_bytes(33, 10, 10, 1) == 0
    assert mtb.mtb_pair_workspace_bytes(0) == 0 and mtb.mtb_pair_workspace_bytes(17) == 0


@pytest.mark.parametrize("w,h,L", [(0, 5, 1), (5, 0, 1), (10, 10, 0), (10, 10, 5), (1 << 16, 1 << 15, 1)])
def test_invalid_sizes_rejected(mtb, w, h, L):
    assert mtb.mtb_pyramid_bytes(w, h, L) == 0
    assert mtb.mtb_bitmaps_bytes(w, h, L) == 0
    from paper_2007_06483_amd import MTBError

    with pytest.raises(MTBError) as e:
        mtb.mtb_get_layout(w, h, L)
    assert e.value.status == 1


# Validation happens before anything touches a device, so these calls pass fake
# (never dereferenced) addresses and must come back with the documented status.
FAKE = ctypes.c_void_p(0x1000)
NULL = None


def _c(mtb):
    return mtb.lib()


def test_build_pyramid_validation(mtb):
    L = _c(mtb)
    need = mtb.mtb_pyramid_bytes(64, 48, 3)
    assert L.mtb_build_pyramid(NULL, 64, 48, 192, 3, FAKE, need, NULL) == 1
    assert L.mtb_build_pyramid(FAKE, 64, 48, 192, 3, NULL, need, NULL) == 1
    assert L.mtb_build_pyramid(FAKE, 64, 48, 191, 3, FAKE, need, NULL) == 1   # stride < 3W
    assert L.mtb_build_pyramid(FAKE, 64, 48, 192, 7, FAKE, need, NULL) == 1   # too many levels
    assert L.mtb_build_pyramid(FAKE, 64, 48, 192, 0, FAKE, need, NULL) == 1
    assert L.mtb_build_pyramid(FAKE, 64, 48, 192, 3, FAKE, need - 1, NULL) == 2


def test_bitmaps_validation(mtb):
    L = _c(mtb)
    need = mtb.mtb_bitmaps_bytes(64, 48, 3)
    assert L.mtb_bitmaps(NULL, 64, 48, 3, 4, FAKE, need, NULL) == 1
    assert L.mtb_bitmaps(FAKE, 64, 48, 3, -1, FAKE, need, NULL) == 1
    assert L.mtb_bitmaps(FAKE, 64, 48, 3, 256, FAKE, need, NULL) == 1
    assert L.mtb_bitmaps(FAKE, 64, 48, 3, 4, FAKE, need - 1, NULL) == 2


def test_align_pair_validation(mtb):
    L = _c(mtb)
    ws = mtb.mtb_pair_workspace_bytes(3)
    args = [FAKE, FAKE, 64, 48, 3, FAKE, ws, FAKE, FAKE, NULL, NULL, NULL]
    for i in (0, 1, 5, 7, 8):
        bad = list(args)
        bad[i] = NULL
        assert L.mtb_align_pair(*bad) == 1, i
    bad = list(args)
    bad[6] = ws - 1
    assert L.mtb_align_pair(*bad) == 2
    bad = list(args)
    bad[4] = 7
    assert L.mtb_align_pair(*bad) == 1


def test_align_stack_validation(mtb):
    L = _c(mtb)
    n = 3
    ptrs = (ctypes.c_void_p * n)(0x1000, 0x2000, 0x3000)
    ws = mtb.mtb_stack_workspace_bytes(n, 64, 48, 3)
    args = [ptrs, n, 64, 48, 192, 3, 4, -1, FAKE, ws, FAKE, FAKE, NULL, NULL]
    assert L.mtb_align_stack(*[NULL if i == 0 else a for i, a in enumerate(args)]) == 1
    for i, v in ((1, 0), (1, 33), (4, 100), (5, 9), (6, -2), (7, 3), (8, NULL), (10, NULL), (11, NULL)):
        bad = list(args)
        bad[i] = v
        assert L.mtb_align_stack(*bad) == 1, (i, v)
    nullp = (ctypes.c_void_p * n)(0x1000, 0, 0x3000)
    bad = list(args)
    bad[0] = nullp
    assert L.mtb_align_stack(*bad) == 1
    bad = list(args)
    bad[9] = ws - 1
    assert L.mtb_align_stack(*bad) == 2


def test_valid_call_without_gpu_is_unsupported(mtb):
    import torch

    if torch.cuda.device_count() > 0:
        pytest.skip("a GPU is visible; this checks the no-device path")
    L = _c(mtb)
    need = mtb.mtb_pyramid_bytes(64, 48, 3)
    assert L.mtb_build_pyramid(FAKE, 64, 48, 192, 3, FAKE, need, NULL) == 4


def _items(mtb, specs):
    from paper_2007_06483_amd import _BatchItem

    arr = (_BatchItem * len(specs))()
    for i, (w, h, L, stride) in enumerate(specs):
        arr[i] = _BatchItem(0x1000 + 0x100 * i, 0x9000 + 0x100 * i, stride, w, h, L, 0)
    return arr


def test_batch_workspace_holds_one_range_per_lane(mtb):
    L = _c(mtb)
    specs = [(64, 48, 3, 192), (32, 24, 2, 96), (64, 48, 3, 192), (64, 48, 3, 256)]
    items = _items(mtb, specs)
    got = L.mtb_batch_workspace_bytes(items, len(specs))
    # Groups: (64x48, stride 192) x2, (32x24) x1, (64x48, stride 256) x1; the
    # three groups run on three lanes, each with a range the size of the
    # largest group's need (at most that of its images as a stack).
    two = mtb.mtb_stack_workspace_bytes(4, 64, 48, 3)
    assert 3 * (mtb.mtb_stack_workspace_bytes(2, 64, 48, 3) - 256) < got <= 3 * two + 4096
    # One group: one range.
    one = L.mtb_batch_workspace_bytes(_items(mtb, [(64, 48, 3, 192)] * 2), 2)
    assert one <= two + 256
    # 17 equal items split into 16 + 1: two lanes, each sized for the 16.
    items17 = _items(mtb, [(64, 48, 3, 192)] * 17)
    items16 = _items(mtb, [(64, 48, 3, 192)] * 16)
    w16 = L.mtb_batch_workspace_bytes(items16, 16)
    assert L.mtb_batch_workspace_bytes(items17, 17) == 2 * (w16 - 256) + 256
    assert w16 > L.mtb_batch_workspace_bytes(items16, 8)
    # At most four lanes: five groups of different sizes take four ranges.
    five = _items(mtb, [(64 + 8 * k, 48, 3, 3 * (64 + 8 * k)) for k in range(5)])
    big = L.mtb_batch_workspace_bytes(_items(mtb, [(96, 48, 3, 288)]), 1)
    assert L.mtb_batch_workspace_bytes(five, 5) == 4 * (big - 256) + 256


def test_batch_validation(mtb):
    L = _c(mtb)
    items = _items(mtb, [(64, 48, 3, 192), (32, 24, 2, 96)])
    ws = L.mtb_batch_workspace_bytes(items, 2)
    assert ws > 0
    assert L.mtb_batch_workspace_bytes(NULL, 2) == 0
    assert L.mtb_batch_workspace_bytes(items, 0) == 0
    args = [items, 2, 4, FAKE, ws, FAKE, FAKE, NULL]
    for i, v in ((0, NULL), (1, 0), (1, 4097), (2, -1), (2, 256), (3, NULL), (5, NULL), (6, NULL)):
        bad = list(args)
        bad[i] = v
        assert L.mtb_align_batch(*bad) == 1, (i, v)
    bad = list(args)
    bad[4] = ws - 1
    assert L.mtb_align_batch(*bad) == 2
    for field, value in (("levels", 7), ("levels", 0), ("row_stride", 95), ("reserved", 1),
                         ("d_ref_rgb", None), ("width", 0)):
        broken = _items(mtb, [(64, 48, 3, 192), (32, 24, 2, 96)])
        setattr(broken[1], field, value)
        assert L.mtb_batch_workspace_bytes(broken, 2) == 0, field
        assert L.mtb_align_batch(broken, 2, 4, FAKE, ws, FAKE, FAKE, NULL) == 1, field


def test_profile_state_machine(mtb):
    L = _c(mtb)
    from paper_2007_06483_amd import _KernelTime

    out = (_KernelTime * 4)()
    cnt = ctypes.c_int32(-1)
    assert L.mtb_profile_pause(1) == 1              # profiling is off
    assert L.mtb_profile_end(out, 4, ctypes.byref(cnt)) == 1
    assert L.mtb_profile_begin(b"x" * 48) == 1      # name too long
    assert L.mtb_profile_begin(b"k_pyramid") == 0
    assert L.mtb_profile_begin(None) == 1           # already on
    assert L.mtb_profile_pause(1) == 0 and L.mtb_profile_pause(0) == 0
    assert L.mtb_profile_end(out, 4, ctypes.byref(cnt)) == 0 and cnt.value == 0
    assert L.mtb_profile_pause(0) == 1


def test_apply_shifts_validation(mtb):
    L = _c(mtb)
    n = 2
    ins = (ctypes.c_void_p * n)(0x1000, 0x2000)
    outs = (ctypes.c_void_p * n)(0x3000, 0x4000)
    args = [ins, n, 64, 48, 192, FAKE, 0, outs, 192, NULL]
    for i, v in ((0, NULL), (1, 0), (1, 33), (2, 0), (3, 0), (4, 191), (5, NULL), (6, 2), (6, -1),
                 (7, NULL), (8, 191)):
        bad = list(args)
        bad[i] = v
        assert L.mtb_apply_shifts(*bad) == 1, (i, v)
    bad = list(args)
    bad[7] = (ctypes.c_void_p * n)(0x3000, 0)
    assert L.mtb_apply_shifts(*bad) == 1


def test_stage_rgb_validation(mtb):
    L = _c(mtb)
    args = [FAKE, 192, 64, 48, FAKE, 256, NULL]
    for i, v in ((0, NULL), (1, 191), (2, 0), (3, 0), (4, NULL), (5, 191)):
        bad = list(args)
        bad[i] = v
        assert L.mtb_stage_rgb(*bad) == 1, (i, v)
    # 2^16 x 2^16 pixels: strides valid, pixel count too large.
    assert L.mtb_stage_rgb(FAKE, 3 << 16, 1 << 16, 1 << 16, FAKE, 3 << 16, NULL) == 1


def test_quadrant_validation(mtb):
    L = _c(mtb)
    ws = L.mtb_quadrant_workspace_bytes(64, 48, 192, 3)
    assert ws > 0
    assert L.mtb_quadrant_workspace_bytes(64, 48, 192, 6) == 0   # too many levels for 32x24 quadrants
    assert L.mtb_quadrant_workspace_bytes(1, 48, 192, 1) == 0
    assert L.mtb_quadrant_workspace_bytes(64, 48, 191, 3) == 0
    args = [FAKE, FAKE, 64, 48, 192, 3, 4, 1, FAKE, ws, FAKE, FAKE, FAKE, NULL]
    for i, v in ((0, NULL), (1, NULL), (2, 1), (3, 1), (4, 100), (5, 6), (6, 256), (7, -1), (8, NULL),
                 (10, NULL), (11, NULL), (12, NULL)):
        bad = list(args)
        bad[i] = v
        assert L.mtb_align_quadrants(*bad) == 1, (i, v)
    bad = list(args)
    bad[9] = ws - 1
    assert L.mtb_align_quadrants(*bad) == 2


def test_stream_probe_validation(mtb):
    L = mtb.lib()
    A, B = ctypes.c_void_p(0x10000), ctypes.c_void_p(0x20000)
    assert L.mtb_probe_stream(None, 1 << 20, B, 0, None) == 1
    assert L.mtb_probe_stream(A, 8, B, 0, None) == 1                      # less than one 16-byte word
    assert L.mtb_probe_stream(A, 1 << 20, B, (1 << 20) + 16, None) == 1  # writes more than it reads
    assert L.mtb_probe_stream(A, 1 << 20, B, 1 << 17, None) == 1          # 8 bytes read per byte written
    assert L.mtb_probe_stream(A, 1 << 20, None, 4096, None) == 1          # writes without a destination
    assert L.mtb_probe_stream(ctypes.c_void_p(0x10004), 1 << 20, B, 0, None) == 1  # misaligned
    assert L.mtb_probe_stream(A, 1 << 20, B, 1 << 18, None) == 4          # valid, but no device here


def _stacks(mtb, specs):
    """Stack items with fake device pointers: specs [(n, w, h, L, stride, ref_index)]."""
    from paper_2007_06483_amd import _BatchStack

    arr = (_BatchStack * len(specs))()
    keep = []
    for i, (n, w, h, L, stride, ref) in enumerate(specs):
        ptrs = (ctypes.c_void_p * n)(*[0x1000 + 0x10000 * i + 0x100 * k for k in range(n)])
        keep.append(ptrs)
        arr[i] = _BatchStack(ctypes.cast(ptrs, ctypes.POINTER(ctypes.c_void_p)), n, ref, stride, w, h, L, 0)
    return arr, keep


def test_stack_batch_workspace_and_validation(mtb):
    L = _c(mtb)
    items, keep = _stacks(mtb, [(3, 64, 48, 3, 192, -1), (5, 32, 24, 2, 96, 0), (1, 64, 48, 3, 192, -1)])
    ws = L.mtb_batch_stacks_workspace_bytes(items, 3)
    assert ws > 0
    # A stack batch of pairs needs what the pair batch of the same pairs needs.
    two, keep2 = _stacks(mtb, [(2, 64, 48, 3, 192, 0), (2, 32, 24, 2, 96, 0)])
    pairs = _items(mtb, [(64, 48, 3, 192), (32, 24, 2, 96)])
    assert L.mtb_batch_stacks_workspace_bytes(two, 2) == L.mtb_batch_workspace_bytes(pairs, 2)
    assert L.mtb_batch_stacks_workspace_bytes(None, 3) == 0
    assert L.mtb_batch_stacks_workspace_bytes(items, 0) == 0
    args = [items, 3, 4, FAKE, ws, FAKE, FAKE, NULL]
    for i, v in ((0, NULL), (1, 0), (1, 4097), (2, -1), (2, 256), (3, NULL), (5, NULL), (6, NULL)):
        bad = list(args)
        bad[i] = v
        assert L.mtb_align_batch_stacks(*bad) == 1, (i, v)
    bad = list(args)
    bad[4] = ws - 1
    assert L.mtb_align_batch_stacks(*bad) == 2
    for field, value in (("n", 0), ("n", 33), ("ref_index", 5), ("ref_index", -2), ("levels", 7),
                         ("row_stride", 95), ("reserved", 1), ("d_rgb", None), ("width", 0)):
        broken, keep3 = _stacks(mtb, [(3, 64, 48, 3, 192, -1), (5, 32, 24, 2, 96, 0)])
        setattr(broken[1], field, value)
        assert L.mtb_batch_stacks_workspace_bytes(broken, 2) == 0, field
        assert L.mtb_align_batch_stacks(broken, 2, 4, FAKE, ws, FAKE, FAKE, NULL) == 1, field
    # A null image pointer inside a stack is refused too.
    holes, keep4 = _stacks(mtb, [(3, 64, 48, 3, 192, -1)])
    keep4[0][1] = None
    assert L.mtb_batch_stacks_workspace_bytes(holes, 1) == 0


def test_level1_from_level0_rule_and_shape(mtb):
    # The built-in rule forms level 1's bitmaps from level 0's gray for launch
    # sets of at least 96 Mi level-0 pixels; a stored shape overrides it.
    mtb.mtb_tune_reset()
    assert mtb.mtb_level1_from_level0(7, 6000, 4000, 18000, 7)          # 168 MP
    assert mtb.mtb_level1_from_level0(8, 4096, 3072, 12288, 6)          # exactly 96 Mi
    assert not mtb.mtb_level1_from_level0(3, 6000, 4000, 18000, 7)      # 72 MP
    assert not mtb.mtb_level1_from_level0(2, 4096, 3072, 12288, 6)
    assert not mtb.mtb_level1_from_level0(32, 6000, 4000, 18000, 1)     # one level: no level 1
    mtb.mtb_set_shape(2, 640, 480, 1920, 5, {"level1_from_level0": 1})
    assert mtb.mtb_level1_from_level0(2, 640, 480, 1920, 5)
    mtb.mtb_set_shape(7, 6000, 4000, 18000, 7, {"level1_from_level0": 0})
    assert not mtb.mtb_level1_from_level0(7, 6000, 4000, 18000, 7)
    mtb.mtb_tune_reset()
    for bad in [(0, 640, 480, 1920, 5), (33, 640, 480, 1920, 5), (2, 640, 480, 1000, 5), (2, 640, 480, 1920, 11)]:
        with pytest.raises(RuntimeError):
            mtb.mtb_level1_from_level0(*bad)
