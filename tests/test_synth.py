"""The seeded input generator: determinism, exact quantisation, saturation and shifts."""

import math

import numpy as np

import synth


def test_same_seed_same_bytes():
    a = synth.make_pair(96, 64, 12, 9, 5)
    b = synth.make_pair(96, 64, 12, 9, 5)
    assert synth.sha256(a[0]) == synth.sha256(b[0])
    assert synth.sha256(a[1]) == synth.sha256(b[1])
    assert a[2] == b[2]
    c = synth.make_pair(96, 64, 12, 10, 5)
    assert synth.sha256(a[0]) != synth.sha256(c[0])


def test_quantisation_matches_its_definition():
    # q = floor(255 v^(1/2.2) + 0.5) exactly: q counts the thresholds v reaches.
    rng = np.random.default_rng(0)
    v = np.concatenate([rng.uniform(0, 1, 20000), synth.THRESHOLDS,
                        np.nextafter(synth.THRESHOLDS, 0), [0.0, 1.0]])
    q = synth._quantise(v)
    want = np.array([sum(1 for t in synth.THRESHOLDS if x >= t) for x in v[:3000]])
    assert np.array_equal(q[:3000], want)
    # At each threshold the code steps up by exactly one.
    k = np.arange(1, 256)
    assert np.array_equal(q[20000:20255], k)
    assert np.array_equal(q[20255:20510], k - 1)
    assert q[-2] == 0 and q[-1] == 255
    # Agrees with the float formula away from the rounding boundaries.
    approx = np.floor(255 * v[:20000] ** (1 / 2.2) + 0.5)
    assert np.array_equal(q[:20000], approx.astype(np.uint8))


def test_translation_is_edge_replicate():
    img = np.arange(5 * 4 * 3, dtype=np.uint8).reshape(5, 4, 3)
    out = synth.translate(img, 1, -2)
    for y in range(5):
        for x in range(4):
            sy = min(max(y + 2, 0), 4)
            sx = min(max(x - 1, 0), 3)
            assert (out[y, x] == img[sy, sx]).all()


def test_saturation_gain_hits_target_fraction():
    n = 5
    imgs, shifts, gain = synth.make_stack(160, 120, n, 30, 7, 0, sat_frac=0.05)
    assert all(s == (0, 0) for s in shifts)
    sat = np.mean([(im == 255).any(axis=2).mean() for im in imgs])
    assert abs(sat - 0.05) < 0.001


def test_stack_reference_unshifted_and_shifts_in_range():
    imgs, shifts, _ = synth.make_stack(64, 48, 7, 10, 8, 9)
    assert shifts[3] == (0, 0)
    assert all(abs(tx) <= 9 and abs(ty) <= 9 for tx, ty in shifts)
    assert all(im.shape == (48, 64, 3) and im.dtype == np.uint8 for im in imgs)


def test_exposures_are_two_stops_apart():
    # Without clipping, doubling the exposure raises the code by the gamma curve: q ~ 255 (2v)^(1/2.2).
    rng = np.random.default_rng(3)
    rad = np.clip(rng.uniform(0.05, 0.2, (3, 8, 8)), 0, 1)
    lo = synth.expose(rad, -1).astype(float)
    hi = synth.expose(rad, 0).astype(float)
    ratio = (hi / 255) ** 2.2 / np.maximum((lo / 255) ** 2.2, 1e-9)
    assert np.all(np.abs(ratio - 2.0) < 0.35)
    assert math.isclose(float(np.median(ratio)), 2.0, rel_tol=0.05)


def test_serve_levels_formula():
    assert synth.serve_levels(1225, 816) == 5       # 1 + floor(log2(816 / 32)) = 5
    assert synth.serve_levels(8485, 5657) == 7      # capped at 7
    assert synth.serve_levels(64, 64) == 2 and synth.serve_levels(63, 100) == 1


def test_serve_requests_fit_the_base_and_are_reproducible():
    reqs = synth.serve_requests(5, 200.0, 2.0, 8704, 5888)
    again = synth.serve_requests(5, 200.0, 2.0, 8704, 5888)
    assert reqs == again
    assert 250 < len(reqs) < 550                    # Poisson(400)
    arr = [r["arrival"] for r in reqs]
    assert arr == sorted(arr) and arr[-1] < 2.0
    for r in reqs:
        W, H, L = r["width"], r["height"], r["levels"]
        R = 1 << (L - 1)
        assert 3 <= r["n"] <= 9 and L == synth.serve_levels(W, H)
        assert 0.9e6 <= W * H <= 48.5e6
        assert r["offsets"][r["n"] // 2] == (0, 0)
        for (dx, dy), e in zip(r["offsets"], r["exposures"]):
            assert -R <= dx <= R and -R <= dy <= R and 0 <= e < 9
            assert 0 <= r["x0"] + dx and r["x0"] + dx + W <= 8704
            assert 0 <= r["y0"] + dy and r["y0"] + dy + H <= 5888
        assert r["exposures"][r["n"] // 2] == 4


def test_serve_crop_is_a_translation():
    base = [np.arange(40 * 30 * 3, dtype=np.int64).reshape(30, 40, 3) + 1000 * e for e in range(9)]
    req = dict(offsets=[(2, -1), (0, 0), (-3, 2)], exposures=[3, 4, 5], x0=10, y0=8, width=12, height=9)
    ref = synth.serve_crop(base, req, 1)
    mov = synth.serve_crop(base, req, 2)
    # aligned[y][x] = mov[y - dy][x - dx] with (dx, dy) = offset equals the reference scene.
    dx, dy = req["offsets"][2]
    for y in range(9):
        for x in range(12):
            if 0 <= y - dy < 9 and 0 <= x - dx < 12:
                assert mov[y - dy, x - dx, 0] - 1000 == ref[y, x, 0]
