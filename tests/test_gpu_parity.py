"""Bit-exact parity of the HIP path (through the C ABI) with the CPU oracle.

Every intermediate is compared element by element: gray levels, histograms,
medians, unpacked threshold/exclusion bitmaps (and their zero padding bits),
per-level candidate errors, per-level shifts, final shifts and errors.  The
method is integer-only, so the tolerance is zero everywhere.
"""

import numpy as np
import pytest

import oracle
import synth
from mtb_decode import bitmaps, gray_levels, histograms, medians, stack_workspace

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mtb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2007_06483_amd as m

    m.lib()
    return m


DEV = "cuda:0"


def _noise(h, w, seed):
    return np.random.default_rng(seed).integers(0, 256, (h, w, 3), dtype=np.uint8)


def _to_dev(img):
    return torch.from_numpy(np.ascontiguousarray(img)).to(DEV)


def _strided_dev(img, extra, offset):
    """Device view of img whose rows are 3W + extra bytes apart, starting offset bytes in."""
    h, w, _ = img.shape
    stride = 3 * w + extra
    buf = np.random.default_rng(99).integers(0, 256, offset + stride * h + 8, dtype=np.uint8)
    rows = buf[offset:offset + stride * h].reshape(h, stride)
    rows[:, :3 * w] = img.reshape(h, 3 * w)
    d = torch.from_numpy(buf).to(DEV)
    return torch.as_strided(d, (h, w, 3), (stride, 3, 1), offset)


def _check_pyramid(mtb, d_img, img, L, exclude=4):
    h, w, _ = img.shape
    lay = mtb.mtb_get_layout(w, h, L)
    pyr = mtb.mtb_build_pyramid(d_img, L)
    bm = mtb.mtb_bitmaps(pyr, w, h, L, exclude)
    torch.cuda.synchronize()
    pyr_h, bm_h = pyr.cpu().numpy(), bm.cpu().numpy()
    want = oracle.pyramid(img, L, exclude)
    for l, g in enumerate(gray_levels(pyr_h, lay)):
        assert np.array_equal(g, want.gray(l)), f"gray level {l}"
    assert np.array_equal(histograms(pyr_h, lay), want.hist)
    assert np.array_equal(medians(bm_h, lay), want.median)
    for l, (t, e, tp, ep) in enumerate(bitmaps(bm_h, lay)):
        assert np.array_equal(t, want.tb(l)), f"T level {l}"
        assert np.array_equal(e, want.eb(l)), f"E level {l}"
        assert not tp.any() and not ep.any(), f"padding bits set at level {l}"
    return pyr, bm


# Sizes: several 64x64 tiles with ragged right/bottom tiles, odd sizes, single rows
# and columns, more than the seven levels fused in one pass, and the largest level count.
SIZES = [
    (512, 384, 5), (641, 479, 7), (130, 70, 7), (1000, 700, 9), (257, 129, 8),
    (1, 97, 1), (97, 1, 1), (3, 5, 1), (5, 3, 2), (64, 64, 7), (65, 63, 6), (2048, 33, 6),
    (300, 4000, 9), (2100, 2050, 12),
]


@pytest.mark.parametrize("w,h,L", SIZES)
def test_pyramid_and_bitmaps_match_oracle(mtb, w, h, L):
    img = _noise(h, w, w * 7 + h)
    _check_pyramid(mtb, _to_dev(img), img, L)


@pytest.mark.parametrize("w,h,L", [(512, 384, 5), (331, 217, 6)])
def test_scene_pyramid_matches_oracle(mtb, w, h, L):
    ref, mov, _ = synth.make_rect_pair(w, h, 30, 5, 10)
    for img in (ref, mov):
        _check_pyramid(mtb, _to_dev(img), img, L)


@pytest.mark.parametrize("extra,offset", [(1, 0), (5, 3), (64, 1), (0, 2)])
def test_pyramid_with_unaligned_rows(mtb, extra, offset):
    img = _noise(77, 133, 42 + extra)
    _check_pyramid(mtb, _strided_dev(img, extra, offset), img, 5)


@pytest.mark.parametrize("extra,offset", [(0, 1), (0, 3), (2, 2), (7, 1), (9, 0), (13, 3)])
def test_pyramid_unaligned_rows_several_tiles(mtb, extra, offset):
    # Rows at every byte alignment (strides not a multiple of 4 give each row
    # its own), over several 64 x 256 tiles with ragged right and bottom tiles.
    img = _noise(200, 611, 7 + extra + offset)
    _check_pyramid(mtb, _strided_dev(img, extra, offset), img, 7)


@pytest.mark.parametrize("exclude", [0, 1, 7, 127, 200, 255])
def test_bitmaps_exclusion_ranges(mtb, exclude):
    # Thresholds m + X + 1 above 255 and m - X below 0 (the band covers the whole range).
    img = _noise(67, 150, 40 + exclude)
    img[:20] = 250
    img[20:30] = 3
    _check_pyramid(mtb, _to_dev(img), img, 4, exclude)
    for val in (0, 255):
        flat = np.full((40, 70, 3), val, np.uint8)
        _check_pyramid(mtb, _to_dev(flat), flat, 3, exclude)


@pytest.mark.parametrize("exclude", [0, 4, 10])
def test_bitmaps_every_threshold_case(mtb, exclude):
    """Medians on both sides of 128 for each of the three thresholds.

    Gray images (equal channels give gray = channel) with values m + [-25, 25]
    have medians near m; m runs from 0 to 255 in small steps so that every
    ordering of max(m - X, 0), m + 1 and m + X + 1 against 128 and 256 occurs.
    """
    rng = np.random.default_rng(4242 + exclude)
    for m in (0, 2, 40, 110, 115, 117, 118, 120, 122, 123, 124, 126, 127, 128, 130, 131,
              132, 133, 137, 138, 139, 180, 244, 245, 250, 251, 254, 255):
        v = np.clip(m + rng.integers(-25, 26, (97, 333)), 0, 255).astype(np.uint8)
        img = np.repeat(v[:, :, None], 3, axis=2)
        _check_pyramid(mtb, _to_dev(img), img, 3, exclude)


def test_saturated_and_flat_images(mtb):
    for val in (0, 255, 128):
        img = np.full((150, 200, 3), val, np.uint8)
        _check_pyramid(mtb, _to_dev(img), img, 6)
    img = _noise(150, 200, 3)
    img[:, :120] = 255
    _check_pyramid(mtb, _to_dev(img), img, 6)


def _check_pair(mtb, ref, mov, L):
    h, w, _ = ref.shape
    want = oracle.align_pair(ref, mov, L)
    pr = mtb.mtb_build_pyramid(_to_dev(ref), L)
    pm = mtb.mtb_build_pyramid(_to_dev(mov), L)
    br = mtb.mtb_bitmaps(pr, w, h, L)
    bmv = mtb.mtb_bitmaps(pm, w, h, L)
    got = mtb.mtb_align_pair(br, bmv, w, h, L, trace=True, level_shifts=True)
    torch.cuda.synchronize()
    assert tuple(got["shift"].cpu().tolist()) == want["shift"]
    assert int(got["err"].cpu()[0]) == want["err"]
    assert np.array_equal(got["trace"].cpu().numpy().astype(np.int64), want["trace"])
    assert np.array_equal(got["level_shifts"].cpu().numpy(), want["level_shifts"])
    return want


@pytest.mark.parametrize("seed", range(4))
def test_align_pair_rect_scenes(mtb, seed):
    ref, mov, t = synth.make_rect_pair(400 + 37 * seed, 300 - 11 * seed, 50, 200 + seed, 25)
    want = _check_pair(mtb, ref, mov, 5)
    assert want["shift"] == (-t[0], -t[1])


def test_align_pair_blob_workload_512x384(mtb):
    (imgs, _, _), = synth.workload("pair_512x384").stacks
    _check_pair(mtb, imgs[0], imgs[1], 5)


@pytest.mark.parametrize("L", [1, 2, 3, 7, 8, 9])
def test_align_pair_level_counts(mtb, L):
    ref, mov, _ = synth.make_rect_pair(700, 520, 60, 300 + L, 40)
    _check_pair(mtb, ref, mov, L)


def test_align_pair_most_levels(mtb):
    # As many levels as the size allows: the coarsest level is 1 x 1, the
    # three coarsest are searched exhaustively and nine more are fine.
    w, h = 1100, 1030
    L = mtb.mtb_max_levels(w, h)
    assert L == 11
    ref, mov, _ = synth.make_rect_pair(w, h, 80, 333, 200)
    _check_pair(mtb, ref, mov, L)


def test_align_pair_degenerate(mtb):
    flat = np.full((96, 128, 3), 77, np.uint8)
    want = _check_pair(mtb, flat, flat, 4)
    assert want["shift"] == (-15, -15) and want["err"] == 0
    ref, _, _ = synth.make_rect_pair(200, 150, 30, 17, 0)
    want = _check_pair(mtb, ref, ref, 5)
    assert want["shift"] == (0, 0)
    _check_pair(mtb, _noise(1, 300, 1), _noise(1, 300, 2), 1)
    _check_pair(mtb, _noise(301, 2, 3), _noise(301, 2, 4), 2)


def _check_stack(mtb, imgs, L, ref_index=None, exclude=4):
    want = oracle.align_stack(imgs, L, ref_index=ref_index, exclude=exclude, threads=4, keep=True)
    d = [_to_dev(im) for im in imgs]
    got = mtb.mtb_align_stack(d, L, exclude_range=exclude,
                              ref_index=-1 if ref_index is None else ref_index, trace=True)
    torch.cuda.synchronize()
    assert np.array_equal(got["shifts"].cpu().numpy(), want["shifts"])
    assert np.array_equal(got["errs"].cpu().numpy().astype(np.int64), want["errs"])
    tr = got["trace"].cpu().numpy().astype(np.int64)
    for k, r in want["pairs"].items():
        assert np.array_equal(tr[k], r["trace"]), f"trace of image {k}"
    assert not tr[want["ref_index"]].any()
    return got, want


@pytest.mark.parametrize("n", [1, 2, 3, 5, 7])
def test_align_stack_matches_oracle(mtb, n):
    imgs, _, _ = synth.make_stack(333, 251, n, 40, 500 + n, 30, sat_frac=0.05)
    _check_stack(mtb, imgs, 6)


def test_align_stack_largest_stack(mtb):
    # The largest stack the library takes (32 images), exposures repeating
    # around the middle; every image against the middle reference.
    n = mtb.MTB_MAX_STACK
    imgs, _, _ = synth.make_stack(160, 96, n, 12, 31, 6, evs=[float(i % 7 - 3) for i in range(n)])
    _check_stack(mtb, imgs, 4)


def test_align_stack_reference_choice_and_exclusion(mtb):
    imgs, _, _ = synth.make_stack(256, 200, 4, 30, 77, 20)
    _check_stack(mtb, imgs, 5, ref_index=0)
    _check_stack(mtb, imgs, 5, ref_index=3, exclude=0)
    _check_stack(mtb, imgs, 5, ref_index=2, exclude=12)


def test_stack_intermediates_match_oracle(mtb):
    imgs, _, _ = synth.make_stack(321, 203, 3, 30, 88, 15, sat_frac=0.05)
    L = 6
    got, want = _check_stack(mtb, imgs, L)
    lay = mtb.mtb_get_layout(321, 203, L)
    ws = got["workspace"]
    pyrs, bms = stack_workspace(mtb, ws, 3, lay)
    # Below the size where the alignment calls form level 1's bitmaps from
    # level 0's gray, level 1's gray is stored like every other level.
    assert not mtb.mtb_level1_from_level0(3, 321, 203, 3 * 321, L)
    for i, p in enumerate(want["pyramids"]):
        for l, g in enumerate(gray_levels(pyrs[i], lay)):
            assert np.array_equal(g, p.gray(l))
        assert np.array_equal(histograms(pyrs[i], lay), p.hist)
        assert np.array_equal(medians(bms[i], lay), p.median)
        for l, (t, e, tp, ep) in enumerate(bitmaps(bms[i], lay)):
            assert np.array_equal(t, p.tb(l)) and np.array_equal(e, p.eb(l))
            assert not tp.any() and not ep.any()


@pytest.mark.parametrize("w,h,L", [(1, 1, 1), (2, 3, 2), (65, 7, 3), (127, 2, 2), (1023, 9, 4),
                                   (1024, 8, 4), (1025, 19, 5), (2049, 33, 6), (3000, 5, 2),
                                   (6000, 17, 3)])
def test_stack_bitmaps_of_two_row_units(mtb, w, h, L):
    # With level1_from_level0 (the built-in rule takes it for large launch
    # sets; forced here) the bitmaps pass forms levels 0 and 1 from level 0's
    # gray in units of two rows by 1024 pixels: odd heights leave a last unit
    # of one row (and no level-1 row), widths off a multiple of 1024 leave
    # lanes past a row's words, and level 1's last padding word can lie past
    # level 0's words.  Every bit, padding included, and every median must be
    # the oracle's; shifts, errors and traces too.
    imgs, _, _ = synth.make_stack(w, h, 2, max(2, w * h // 4000), 900 + w + h, min(3, w // 4, h // 4),
                                  sat_frac=0.05)
    mtb.mtb_tune_reset()
    mtb.mtb_set_shape(2, w, h, 3 * w, L, {"level1_from_level0": 1})
    assert mtb.mtb_level1_from_level0(2, w, h, 3 * w, L) == (L >= 2)
    try:
        got, want = _check_stack(mtb, imgs, L)
    finally:
        mtb.mtb_tune_reset()
    lay = mtb.mtb_get_layout(w, h, L)
    pyrs, bms = stack_workspace(mtb, got["workspace"], 2, lay)
    for i, p in enumerate(want["pyramids"]):
        assert np.array_equal(medians(bms[i], lay), p.median), f"medians of image {i}"
        for l, (t, e, tp, ep) in enumerate(bitmaps(bms[i], lay)):
            assert np.array_equal(t, p.tb(l)) and np.array_equal(e, p.eb(l)), f"image {i} level {l}"
            assert not tp.any() and not ep.any(), f"padding bits of image {i} level {l}"


@pytest.mark.parametrize("w,h,n", [(2048, 1536, 2), (2100, 1700, 1), (1300, 1100, 2)])
def test_stack_histograms_many_workgroups_per_image(mtb, w, h, n):
    # Launches with a few hundred pyramid workgroups per image (the first two
    # cases) merge the histograms through per-XCD copies and tile tickets;
    # the third stays below that and adds into the histograms directly.
    # Both must give the oracle's histograms, medians and shifts.
    imgs, _, _ = synth.make_stack(w, h, n, 40, 700 + w + n, 20, sat_frac=0.05)
    L = 6
    got, want = _check_stack(mtb, imgs, L)
    blocks, merged = mtb.mtb_test_last_pyramid()
    assert merged == ((w, h) != (1300, 1100)), (blocks, merged)
    lay = mtb.mtb_get_layout(w, h, L)
    pyrs, bms = stack_workspace(mtb, got["workspace"], n, lay)
    for i, p in enumerate(want["pyramids"]):
        assert np.array_equal(histograms(pyrs[i], lay), p.hist), f"histograms of image {i}"
        assert np.array_equal(medians(bms[i], lay), p.median), f"medians of image {i}"


def test_repeated_runs_are_bit_identical(mtb):
    imgs, _, _ = synth.make_stack(800, 600, 5, 60, 91, 40, sat_frac=0.05)
    d = [_to_dev(im) for im in imgs]
    a = mtb.mtb_align_stack(d, 7, trace=True)
    b = mtb.mtb_align_stack(d, 7, trace=True)
    torch.cuda.synchronize()
    assert torch.equal(a["shifts"], b["shifts"]) and torch.equal(a["errs"], b["errs"])
    assert torch.equal(a["trace"], b["trace"])
    lay = mtb.mtb_get_layout(800, 600, 7)
    n = 5
    # Compare every defined byte of the pyramids and bitmaps (row padding and the
    # gaps between aligned planes hold no defined value).
    pa, ba = stack_workspace(mtb, a["workspace"], n, lay)
    pb, bb = stack_workspace(mtb, b["workspace"], n, lay)
    for i in range(n):
        for ga, gb in zip(gray_levels(pa[i], lay), gray_levels(pb[i], lay)):
            assert np.array_equal(ga, gb)
        assert np.array_equal(histograms(pa[i], lay), histograms(pb[i], lay))
        assert np.array_equal(medians(ba[i], lay), medians(bb[i], lay))
        for l in range(lay.levels):
            for off in (lay.tb_offset[l], lay.eb_offset[l]):
                size = 8 * lay.words_per_row[l] * lay.level_height[l]
                assert np.array_equal(ba[i][off:off + size], bb[i][off:off + size])


@pytest.mark.timeout(900)
def test_full_size_pair_4096x3072(mtb):
    w = synth.workload("pair_4096x3072")
    (imgs, _, _), = w.stacks
    _check_stack(mtb, imgs, w.levels, ref_index=0)


@pytest.mark.timeout(1200)
def test_full_size_stack_7x6000x4000(mtb):
    w = synth.workload("stack7_6000x4000")
    (imgs, _, ref), = w.stacks
    _check_stack(mtb, imgs, w.levels, ref_index=ref)


def test_small_pair_search_is_one_launch(mtb):
    # A 512x384 pair's two bitmap pyramids fit one workgroup's LDS: the
    # search is a single launch with no zeroed state, and every level's nine
    # errors still equal the oracle's.
    (imgs, _, _), = synth.workload("pair_512x384").stacks
    ref, mov = imgs
    h, w, _ = ref.shape
    br = mtb.mtb_bitmaps(mtb.mtb_build_pyramid(_to_dev(ref), 5), w, h, 5)
    bmv = mtb.mtb_bitmaps(mtb.mtb_build_pyramid(_to_dev(mov), 5), w, h, 5)
    torch.cuda.synchronize()
    mtb.mtb_profile_begin(None)
    mtb.mtb_align_pair(br, bmv, w, h, 5)
    torch.cuda.synchronize()
    launches = {k: c for k, (c, _) in mtb.mtb_profile_end().items()}
    assert launches == {"k_search_small": 1}, launches
    _check_pair(mtb, ref, mov, 5)


# Sizes on both sides of the one-workgroup search's LDS limit (144 KiB for
# both pyramids' planes), odd widths and heights, one-row and one-column
# images, and the most levels the size allows.
@pytest.mark.parametrize("w,h,L", [(512, 384, 5), (530, 380, 6), (600, 420, 4), (129, 97, 7), (1000, 100, 3),
                                   (2000, 40, 6), (37, 600, 5), (1, 500, 1), (700, 1, 1), (64, 64, 7)])
def test_one_workgroup_search_equals_launch_chain(mtb, w, h, L):
    # Stacks of three: the one-workgroup search (the rule, where it fits) and
    # the coarse and fine launches (small_search 0) give identical shifts,
    # errors and traces, equal to the oracle's.
    imgs, _, _ = synth.make_stack(w, h, 3, 12, 900 + w + h, min(w, h) // 4, sat_frac=0.05)
    d = [_to_dev(im) for im in imgs]
    mtb.mtb_tune_reset()
    got = mtb.mtb_align_stack(d, L, trace=True)
    mtb.mtb_set_shape(3, w, h, 3 * w, L, {"small_search": 0})
    alt = mtb.mtb_align_stack(d, L, trace=True)
    torch.cuda.synchronize()
    mtb.mtb_tune_reset()
    for k in ("shifts", "errs", "trace"):
        assert np.array_equal(got[k].cpu().numpy(), alt[k].cpu().numpy()), k
    want = oracle.align_stack(imgs, L, threads=4, keep=False)
    assert np.array_equal(got["shifts"].cpu().numpy(), want["shifts"])
    assert np.array_equal(got["errs"].cpu().numpy().astype(np.int64), want["errs"])
