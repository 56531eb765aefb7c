"""Pins for the CPU oracle: each test checks it against something other than itself.

Hand-worked values, closed forms, invariants, library routines (bincount,
partition) and brute force on tiny inputs.  Each test names the step of the
method it pins (Section III-A / III-B of the paper) and the mistake it would
catch.  None of these tests need a GPU.
"""

import itertools

import numpy as np
import pytest

import oracle
import synth


def _rgb(pixels):
    """(H, W, 3) uint8 image from nested lists of (R, G, B)."""
    return np.array(pixels, dtype=np.uint8)


# ---------------------------------------------------------------- gray (Section III-A)

def test_gray_hand_values():
    # Ward's weights 54/183/19 out of 256, worked by hand:
    # 54*255/256 = 53.79 -> 53, 183*255/256 = 182.29 -> 182, 19*255/256 = 18.93 -> 18.
    # A channel-order or weight mistake changes at least one of these.
    img = _rgb([[(255, 0, 0), (0, 255, 0), (0, 0, 255), (255, 255, 255), (0, 0, 0)]])
    assert oracle.gray(img).tolist() == [[53, 182, 18, 255, 0]]
    # (10, 20, 30): 540 + 3660 + 570 = 4770; 4770 / 256 = 18.63 -> 18.
    assert oracle.gray(_rgb([[(10, 20, 30)]])).tolist() == [[18]]


def test_gray_of_gray_is_identity():
    # The weights sum to 256, so a neutral pixel keeps its value (a wrong shift or sum breaks it).
    v = np.arange(256, dtype=np.uint8)
    img = np.stack([v, v, v], axis=-1)[None]
    assert oracle.gray(img)[0].tolist() == list(range(256))


def test_gray_all_triples_exhaustive():
    # All 2^24 (R, G, B) triples against the floor of the weighted mean.
    r, g, b = np.meshgrid(np.arange(256), np.arange(256), np.arange(256), indexing="ij")
    img = np.stack([r, g, b], axis=-1).astype(np.uint8).reshape(4096, 4096, 3)
    want = ((54 * r.astype(np.int64) + 183 * g + 19 * b) // 256).reshape(4096, 4096)
    assert np.array_equal(oracle.gray(img), want.astype(np.uint8))


def test_gray_monotone_in_each_channel():
    rng = np.random.default_rng(0)
    img = rng.integers(0, 255, (64, 64, 3), dtype=np.uint8)
    base = oracle.gray(img).astype(int)
    for c in range(3):
        up = img.copy()
        up[:, :, c] += 1
        assert (oracle.gray(up).astype(int) >= base).all()


def test_gray_honours_row_stride():
    rng = np.random.default_rng(1)
    img = rng.integers(0, 256, (7, 5, 3), dtype=np.uint8)
    padded = rng.integers(0, 256, (7, 5 * 3 + 13), dtype=np.uint8)
    padded[:, :15] = img.reshape(7, 15)
    view = padded[:, :15].reshape(7, 5, 3)  # strided view: rows 28 bytes apart
    assert view.strides[0] == 28
    assert np.array_equal(oracle.gray(view), oracle.gray(img))


# ---------------------------------------------------------------- pyramid (Section III-A, Fig. 2)

def test_downsample_hand_example():
    g = np.arange(16, dtype=np.uint8).reshape(4, 4)
    # Block sums 10, 18, 42, 50 -> floor means 2, 4, 10, 12.
    assert oracle.downsample(g).tolist() == [[2, 4], [10, 12]]


def test_downsample_floors_not_rounds():
    # (1+2+2+2)/4 = 1.75: floor 1 (rounding would give 2).
    assert oracle.downsample(np.array([[1, 2], [2, 2]], np.uint8)).tolist() == [[1]]
    assert oracle.downsample(np.array([[255, 255], [255, 254]], np.uint8)).tolist() == [[254]]


def test_downsample_drops_odd_edge():
    rng = np.random.default_rng(2)
    g = rng.integers(0, 256, (9, 11), dtype=np.uint8)
    d = oracle.downsample(g)
    assert d.shape == (4, 5)
    g2 = g.copy()
    g2[8, :] = rng.integers(0, 256, 11)
    g2[:, 10] = rng.integers(0, 256, 9)
    assert np.array_equal(oracle.downsample(g2), d)


def test_pyramid_is_recursive_not_block_mean():
    # Three 2x2 blocks summing to 7 and one to 11 give level 1 = [[1,1],[1,2]] and level 2 =
    # (1+1+1+2)>>2 = 1, while the floor mean of the 16 pixels is 32/16 = 2.
    a = np.array([[1, 2], [2, 2]])
    b = np.array([[2, 3], [3, 3]])
    g = np.block([[a, a], [a, b]]).astype(np.uint8)
    img = np.stack([g, g, g], axis=-1)
    p = oracle.pyramid(img, 3)
    assert p.gray(1).tolist() == [[1, 1], [1, 2]]
    assert p.gray(2).tolist() == [[1]]


def test_pyramid_dims_and_constant_image():
    img = np.full((37, 53, 3), 77, np.uint8)
    L = oracle.max_levels(53, 37)
    assert L == 6  # 37 >> 5 = 1, 37 >> 6 = 0
    p = oracle.pyramid(img, L)
    for l in range(L):
        assert p.gray(l).shape == (37 >> l, 53 >> l)
        assert (p.gray(l) == 77).all()
        assert p.median[l] == 77
        assert p.hist[l][77] == (37 >> l) * (53 >> l)


# ---------------------------------------------------------------- histogram and median (Section III-B)

def test_histogram_matches_bincount():
    rng = np.random.default_rng(3)
    g = rng.integers(0, 256, (123, 77), dtype=np.uint8)
    h = oracle.histogram(g)
    assert np.array_equal(h, np.bincount(g.ravel(), minlength=256))
    assert h.sum() == g.size


def test_median_hand_examples():
    def med(vals):
        g = np.array(vals, np.uint8)
        return oracle.median(oracle.histogram(g), g.size)

    assert med([1, 2, 3, 4]) == 2       # lower median of an even count
    assert med([5]) == 5
    assert med([0, 255]) == 0
    assert med([3, 3, 3]) == 3
    assert med([9, 1, 5]) == 5
    assert med([200, 10, 10, 200, 200]) == 200


@pytest.mark.parametrize("n", [1, 2, 3, 10, 255, 256, 1000, 4097])
def test_median_is_lower_order_statistic(n):
    rng = np.random.default_rng(n)
    g = rng.integers(0, 256, n, dtype=np.uint8)
    k = (n - 1) // 2
    assert oracle.median(oracle.histogram(g), n) == int(np.partition(g, k)[k])


# ---------------------------------------------------------------- bitmaps (Sections III-A, III-B)

def test_bitmap_threshold_and_exclusion_boundaries():
    m = 100
    g = np.arange(m - 6, m + 7, dtype=np.uint8)  # 94 .. 106
    t, e = oracle.bitmaps(g, m, 4)
    # Threshold: at or below the median -> 0.
    assert t.tolist() == [0] * 7 + [1] * 6
    # Exclusion: values within +-4 of the median (96..104) are excluded, m+-5 kept.
    assert e.tolist() == [1, 1] + [0] * 9 + [1, 1]


def test_threshold_popcount_at_most_half():
    rng = np.random.default_rng(4)
    for n in (1, 2, 7, 64, 1001):
        g = rng.integers(0, 256, n, dtype=np.uint8)
        if n % 2:
            g[: n // 2] = 17  # ties at the median
        m = oracle.median(oracle.histogram(g), n)
        t, e = oracle.bitmaps(g, m, 4)
        assert int(t.sum()) <= n // 2
        assert np.array_equal(e == 0, np.abs(g.astype(int) - m) <= 4)


# ---------------------------------------------------------------- shifted error (Sections III-A, III-B)

def _shifted(b, cx, cy):
    """Zero-filled shift by padded slicing: out[y][x] = b[y - cy][x - cx]."""
    h, w = b.shape
    pad = np.zeros((h + 2 * abs(cy) + 2 * h, w + 2 * abs(cx) + 2 * w), b.dtype)
    oy, ox = abs(cy) + h, abs(cx) + w
    pad[oy:oy + h, ox:ox + w] = b
    return pad[oy - cy:oy - cy + h, ox - cx:ox - cx + w]


def _brute_error(tr, er, tm, em, cx, cy):
    return int(((tr ^ _shifted(tm, cx, cy)) & er & _shifted(em, cx, cy)).sum())


def test_shift_error_hand_example():
    # Reference T = 1 everywhere, E = 1 everywhere; moving T = 0, E = 1 on a 3x3 grid.
    one = np.ones((3, 3), np.uint8)
    zero = np.zeros((3, 3), np.uint8)
    assert oracle.shift_error(one, one, zero, one, 0, 0) == 9
    # Shifted by (1, 0): column 0 is filled with zeros (E = 0), 6 pixels remain.
    assert oracle.shift_error(one, one, zero, one, 1, 0) == 6
    # Shifted by (-1, -2): overlap is 2 columns x 1 row.
    assert oracle.shift_error(one, one, zero, one, -1, -2) == 2
    # Fully shifted out.
    assert oracle.shift_error(one, one, zero, one, 3, 0) == 0


def test_shift_error_brute_force_all_shifts():
    rng = np.random.default_rng(5)
    for h, w in ((5, 7), (8, 8), (13, 6), (1, 9)):
        tr, er, tm, em = (rng.integers(0, 2, (h, w), dtype=np.uint8) for _ in range(4))
        for cx in range(-w - 1, w + 2):
            for cy in range(-h - 1, h + 2):
                assert oracle.shift_error(tr, er, tm, em, cx, cy) == _brute_error(tr, er, tm, em, cx, cy)


def test_shift_error_symmetry_and_self():
    rng = np.random.default_rng(6)
    ta, ea, tb, eb = (rng.integers(0, 2, (11, 9), dtype=np.uint8) for _ in range(4))
    for cx, cy in itertools.product(range(-4, 5), range(-4, 5)):
        assert oracle.shift_error(ta, ea, tb, eb, cx, cy) == oracle.shift_error(tb, eb, ta, ea, -cx, -cy)
    assert oracle.shift_error(ta, ea, ta, ea, 0, 0) == 0


# ---------------------------------------------------------------- coarse-to-fine search (Section III-A)

def _first_min(surface):
    """Argmin of a 3x3 surface indexed [dy+1][dx+1], lowest (dy, dx) first."""
    best = None
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            v = surface[dy + 1][dx + 1]
            if best is None or v < best[0]:
                best = (v, dx, dy)
    return best


def test_single_level_is_exhaustive_argmin():
    rng = np.random.default_rng(7)
    for seed in range(6):
        ref = rng.integers(0, 256, (23, 31, 3), dtype=np.uint8)
        mov = rng.integers(0, 256, (23, 31, 3), dtype=np.uint8)
        r = oracle.align_pair(ref, mov, 1)
        pr, pm = r["ref"], r["mov"]
        surf = [[_brute_error(pr.tb(0), pr.eb(0), pm.tb(0), pm.eb(0), dx, dy) for dx in (-1, 0, 1)]
                for dy in (-1, 0, 1)]
        v, dx, dy = _first_min(surf)
        assert r["shift"] == (dx, dy)
        assert r["err"] == v
        assert r["trace"][0].reshape(3, 3).tolist() == surf


def test_trace_matches_brute_force_surface_every_level():
    ref, mov, _ = synth.make_rect_pair(96, 64, 25, 11, 6)
    L = 4
    r = oracle.align_pair(ref, mov, L)
    pr, pm = r["ref"], r["mov"]
    base = (0, 0)
    for l in range(L - 1, -1, -1):
        surf = [[_brute_error(pr.tb(l), pr.eb(l), pm.tb(l), pm.eb(l), base[0] + dx, base[1] + dy)
                 for dx in (-1, 0, 1)] for dy in (-1, 0, 1)]
        assert r["trace"][l].reshape(3, 3).tolist() == surf
        v, dx, dy = _first_min(surf)
        s = (base[0] + dx, base[1] + dy)
        assert tuple(r["level_shifts"][l]) == s
        base = (2 * s[0], 2 * s[1])
    assert r["shift"] == tuple(r["level_shifts"][0])


def test_flat_image_takes_lowest_candidate_everywhere():
    # All errors are 0, so the first candidate (-1, -1) wins at every level and the
    # offsets compound to (-(2^L - 1), -(2^L - 1)).
    img = np.full((64, 64, 3), 128, np.uint8)
    for L in (1, 3, 5):
        r = oracle.align_pair(img, img, L)
        R = 2 ** L - 1
        assert r["shift"] == (-R, -R)
        assert r["err"] == 0


def test_self_alignment_is_zero():
    ref, _, _ = synth.make_rect_pair(160, 120, 40, 12, 0)
    r = oracle.align_pair(ref, ref, 5)
    assert r["shift"] == (0, 0)
    assert r["err"] == 0
    assert (r["level_shifts"] == 0).all()
    # Candidate (0, 0) (index 4) has zero error at every level.
    assert (r["trace"][:, 4] == 0).all()


@pytest.mark.parametrize("seed", range(8))
def test_planted_translation_is_recovered(seed):
    ref, mov, (tx, ty) = synth.make_rect_pair(256, 192, 60, 100 + seed, 20)
    r = oracle.align_pair(ref, mov, 5)
    assert r["shift"] == (-tx, -ty)


def test_search_reaches_exhaustive_minimum_on_tiny_planted_images():
    # With a unique exhaustive level-0 minimum the pyramid search lands on it.
    ref, mov, (tx, ty) = synth.make_rect_pair(64, 48, 20, 21, 3)
    L = 3
    r = oracle.align_pair(ref, mov, L)
    pr, pm = r["ref"], r["mov"]
    R = 2 ** L - 1
    surf = {(cx, cy): _brute_error(pr.tb(0), pr.eb(0), pm.tb(0), pm.eb(0), cx, cy)
            for cx in range(-R, R + 1) for cy in range(-R, R + 1)}
    best = min(surf.values())
    winners = [c for c, v in surf.items() if v == best]
    assert len(winners) == 1
    assert r["shift"] == winners[0] == (-tx, -ty)


def test_cfg1_pair_brute_force_level0_surface():
    """The 512x384 pair workload (40 blobs, 2^0 / 2^-2, 5 levels, shift range +-31):
    its level-0 error over every shift in [-31, 31]^2, counted by padded slicing
    (not the oracle's shift routine), has its minimum where the oracle's search
    ends, and the oracle's level-0 error equals that minimum.

    On this input the minimum (0) is reached by eight shifts, the planted answer
    (-9, 4) among them: the threshold edges of the smooth blobs lie inside the
    +-4 exclusion band, so no one-pixel move changes a counted pixel there, and
    the tie-break picks the lowest (dy, dx) of the candidates the pyramid reaches.
    """
    w = synth.workload("pair_512x384")
    (imgs, shifts, _), = w.stacks
    r = oracle.align_pair(imgs[0], imgs[1], w.levels)
    pr, pm = r["ref"], r["mov"]
    R = 2 ** w.levels - 1
    tr, er, tm, em = pr.tb(0), pr.eb(0), pm.tb(0), pm.eb(0)
    surf = {(cx, cy): _brute_error(tr, er, tm, em, cx, cy)
            for cy in range(-R, R + 1) for cx in range(-R, R + 1)}
    best = min(surf.values())
    assert r["err"] == best
    assert surf[r["shift"]] == best
    zero_set = sorted((c for c, v in surf.items() if v == best), key=lambda c: (c[1], c[0]))
    planted = (-shifts[1][0], -shifts[1][1])
    assert planted in zero_set
    assert r["shift"] == zero_set[0] == (-10, 3)
    assert len(zero_set) == 8


# ---------------------------------------------------------------- stacks (Section III-B)

def test_stack_is_independent_pairs_against_reference():
    imgs, shifts, _ = synth.make_stack(96, 64, 5, 12, 31, 6)
    out = oracle.align_stack(imgs, 4, threads=3)
    assert out["ref_index"] == 2
    assert tuple(out["shifts"][2]) == (0, 0) and out["errs"][2] == 0
    for k in (0, 1, 3, 4):
        r = oracle.align_pair(imgs[2], imgs[k], 4)
        assert tuple(out["shifts"][k]) == r["shift"]
        assert out["errs"][k] == r["err"]


def test_stack_permutation_of_moving_images():
    imgs, _, _ = synth.make_stack(80, 48, 5, 10, 32, 5)
    a = oracle.align_stack(imgs, 3)
    perm = [4, 3, 2, 1, 0]  # the middle (reference) stays in place
    b = oracle.align_stack([imgs[p] for p in perm], 3)
    assert np.array_equal(b["shifts"], a["shifts"][perm])
    assert np.array_equal(b["errs"], a["errs"][perm])


def test_stack_threads_do_not_change_results():
    imgs, _, _ = synth.make_stack(64, 48, 4, 10, 33, 4)
    a = oracle.align_stack(imgs, 3, threads=1)
    b = oracle.align_stack(imgs, 3, threads=4)
    assert np.array_equal(a["shifts"], b["shifts"]) and np.array_equal(a["errs"], b["errs"])


# ---- applying the shift (Section III-B): two fill readings, pinned to an
# independent translation (the generator's edge-replicate slicing) and to
# properties of a translation.

def test_apply_shift_edge_fill_equals_independent_translation():
    rng = np.random.default_rng(17)
    for H, W in ((1, 1), (1, 9), (7, 1), (13, 17), (40, 33)):
        img = rng.integers(0, 256, (H, W, 3), dtype=np.uint8)
        for dx in (-W - 3, -W, -5, -1, 0, 1, 4, W - 1, W + 2):
            for dy in (-H - 1, -2, 0, 3, H):
                assert np.array_equal(oracle.apply_shift(img, dx, dy, 1), synth.translate(img, dx, dy)), (H, W, dx, dy)


def test_apply_shift_zero_fill_is_edge_fill_inside_and_zero_outside():
    rng = np.random.default_rng(18)
    img = rng.integers(1, 256, (21, 30, 3), dtype=np.uint8)   # no zero bytes in the image
    for dx, dy in ((0, 0), (3, -2), (-7, 5), (29, 20), (-31, 0), (0, 21)):
        z = oracle.apply_shift(img, dx, dy, 0)
        e = oracle.apply_shift(img, dx, dy, 1)
        ys, xs = np.mgrid[0:21, 0:30]
        inside = (ys - dy >= 0) & (ys - dy < 21) & (xs - dx >= 0) & (xs - dx < 30)
        assert np.array_equal(z[inside], e[inside])
        assert not z[~inside].any()
        assert int(inside.sum()) == max(0, 21 - abs(dy)) * max(0, 30 - abs(dx))


def test_apply_shift_undoes_a_translation_and_ignores_row_padding():
    rng = np.random.default_rng(19)
    img = rng.integers(0, 256, (50, 64, 3), dtype=np.uint8)
    assert np.array_equal(oracle.apply_shift(img, 0, 0, 0), img)
    tx, ty = 6, -4
    moved = synth.translate(img, tx, ty)
    back = oracle.apply_shift(moved, -tx, -ty, 0)
    # back[y][x] = moved[y + ty][x + tx] = img[y][x] wherever that stays in the image.
    assert np.array_equal(back[-ty:50, 0:64 - tx], img[-ty:50, 0:64 - tx])
    assert not back[:-ty].any() and not back[:, 64 - tx:].any()
    padded = np.zeros((50, 64 + 5, 3), np.uint8)
    padded[:, :64] = moved
    assert np.array_equal(oracle.apply_shift(padded[:, :64], -tx, -ty, 1), oracle.apply_shift(moved, -tx, -ty, 1))


# ---- chained stacks: pairwise along the exposure order, shifts summed.

def test_chained_two_images_is_the_pair():
    ref, mov, _ = synth.make_rect_pair(160, 120, 12, 31, 6)
    ch = oracle.align_stack_chained([ref, mov], 4, ref_index=0)
    direct = oracle.align_pair(ref, mov, 4)
    assert tuple(ch["shifts"][1]) == direct["shift"] and ch["errs"][1] == direct["err"]


def test_chained_sums_planted_translations():
    # One exposure of a sharp scene, each image translated by its own planted
    # shift: neighbours differ by t_k - t_{k+1}, and the summed chain must give
    # every image's shift against the reference, -(t_k - t_ref).
    rng = np.random.default_rng(32)
    rad = synth.rect_field(240, 180, 30, rng)
    base = synth.expose(rad, 0.0)
    planted = [(5, -3), (-2, 4), (0, 0), (6, 1), (-4, -6)]
    imgs = [synth.translate(base, tx, ty) for tx, ty in planted]
    ch = oracle.align_stack_chained(imgs, 5, ref_index=2)
    direct = oracle.align_stack(imgs, 5, ref_index=2)
    want = np.array([(-(tx - 0), -(ty - 0)) for tx, ty in planted], np.int32)
    assert np.array_equal(direct["shifts"], want)
    assert np.array_equal(ch["shifts"], want)
    assert ch["errs"][2] == 0 and tuple(ch["shifts"][2]) == (0, 0)


# ---- quadrant check (Section II): quadrants agree under a translation and
# disagree under a rotation.

def _rotate_nearest(img, degrees):
    """Nearest-neighbour rotation about the image centre (edge pixels repeated)."""
    H, W = img.shape[:2]
    t = np.deg2rad(degrees)
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    cy, cx = (H - 1) / 2.0, (W - 1) / 2.0
    sx = np.cos(t) * (xs - cx) + np.sin(t) * (ys - cy) + cx
    sy = -np.sin(t) * (xs - cx) + np.cos(t) * (ys - cy) + cy
    sx = np.clip(np.rint(sx), 0, W - 1).astype(np.int64)
    sy = np.clip(np.rint(sy), 0, H - 1).astype(np.int64)
    return img[sy, sx]


def test_quadrants_split_and_agree_under_translation():
    q = oracle.quadrants(np.zeros((7, 9, 3), np.uint8))
    assert [a.shape[:2] for a in q] == [(3, 4), (3, 5), (4, 4), (4, 5)]
    rng = np.random.default_rng(41)
    base = synth.expose(synth.rect_field(480, 360, 60, rng), 0.0)
    moved = synth.translate(base, 5, -3)
    r = oracle.align_quadrants(base, moved, 5)
    assert (r["shifts"] == np.array([-5, 3])).all() and r["flag"] == 0


def test_quadrants_flag_a_rotation():
    rng = np.random.default_rng(42)
    base = synth.expose(synth.rect_field(480, 360, 60, rng), 0.0)
    rot = _rotate_nearest(base, 3.0)
    r = oracle.align_quadrants(base, rot, 5)
    # A rotation about the centre moves the quadrants in different directions.
    assert r["flag"] == 1
    assert len({tuple(s) for s in r["shifts"]}) > 1
