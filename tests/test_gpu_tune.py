"""Launch shapes never change results: the tuner's choice and explicit shapes
(pyramid and bitmap grids from a quarter to four rounds, pyramid tile groups
of 1, 2 and 4, 2 to 8 wavefronts per bitmaps workgroup, 0 to 5 exhaustive
coarse levels, every fine level's rows per stream from 4 to 64 and stream
widths of 8 to 64 lanes) give bit-identical shifts, errors and traces, equal
to the oracle's.  Tuned shapes survive a save and load; batch groups are
tuned and use their shapes."""

import os

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

DEV = "cuda:0"


@pytest.fixture(scope="module")
def mtb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2007_06483_amd as m

    m.lib()
    m.mtb_tune_reset()
    yield m
    m.mtb_tune_reset()


def _stack(n, w, h, seed, shift):
    imgs, _, _ = synth.make_stack(w, h, n, 30, seed, shift, sat_frac=0.05)
    return imgs, [torch.from_numpy(im).to(DEV) for im in imgs]


def _run(mtb, d, L):
    r = mtb.mtb_align_stack(d, L, trace=True)
    torch.cuda.synchronize()
    return r["shifts"].cpu().numpy(), r["errs"].cpu().numpy(), r["trace"].cpu().numpy()


def test_tuned_shape_keeps_results_and_is_stored(mtb):
    imgs, d = _stack(5, 900, 640, 61, 25)
    L = 6
    before = _run(mtb, d, L)
    shape = mtb.mtb_tune_stack(d, L)
    assert 25 <= shape["pyramid_slots_pct"] <= 400 and 25 <= shape["bitmaps_blocks_pct"] <= 100
    assert shape["pyramid_tile_group"] in (1, 2, 4) and shape["bitmaps_waves"] in (2, 4, 8)
    assert -1 <= shape["coarse_levels"] <= 5
    assert all(w in (0, 8, 16, 32, 64) for w in shape["search_lanes"])
    assert all(r == 0 or (r % 4 == 0 and 4 <= r <= 64) for r in shape["search_rows"])
    assert shape["step_ms"] > 0 and shape["default_ms"] > 0
    assert shape["step_ms"] <= shape["default_ms"]
    stored = mtb.mtb_tuned_shape(5, 900, 640, 2700, L)
    assert stored is not None
    keys = ("pyramid_slots_pct", "pyramid_tile_group", "bitmaps_blocks_pct", "bitmaps_waves", "coarse_levels",
            "small_search", "level1_from_level0", "search_rows", "search_lanes")
    assert {k: stored[k] for k in keys} == {k: shape[k] for k in keys}
    after = _run(mtb, d, L)
    for a, b in zip(before, after):
        assert np.array_equal(a, b)
    want = oracle.align_stack(imgs, L, threads=4)
    assert np.array_equal(after[0], want["shifts"])
    assert np.array_equal(after[1].astype(np.int64), want["errs"])


@pytest.mark.parametrize("pyr,grp,bm,waves,coarse,l1", [(25, 1, 25, 2, -1, 1), (50, 2, 100, 8, 0, 1),
                                                       (200, 4, 50, 4, 3, 0), (400, 1, 100, 8, 1, 0),
                                                       (100, 4, 75, 2, 2, 1), (100, 1, 100, 4, 4, 1),
                                                       (100, 2, 100, 4, 5, -1)])
def test_explicit_shapes_give_identical_results(mtb, pyr, grp, bm, waves, coarse, l1):
    imgs, d = _stack(4, 1100, 700, 62, 30)
    L = 6
    mtb.mtb_tune_reset()
    ref = _run(mtb, d, L)
    want = oracle.align_stack(imgs, L, threads=4)
    assert np.array_equal(ref[0], want["shifts"])
    for rows, lanes in ((4, 8), (8, 64), (28, 16), (64, 32), (12, 0)):
        mtb.mtb_set_shape(4, 1100, 700, 3300, L, {"pyramid_slots_pct": pyr, "pyramid_tile_group": grp,
                                                  "bitmaps_blocks_pct": bm, "bitmaps_waves": waves,
                                                  "coarse_levels": coarse, "level1_from_level0": l1,
                                                  "search_rows": [rows] * 16, "search_lanes": [lanes] * 16})
        assert mtb.mtb_level1_from_level0(4, 1100, 700, 3300, L) == (l1 == 1)
        got = _run(mtb, d, L)
        for a, b in zip(ref, got):
            assert np.array_equal(a, b), (pyr, grp, bm, waves, coarse, l1, rows, lanes)
    mtb.mtb_tune_reset()


def test_tuned_shapes_survive_save_and_load(mtb, tmp_path):
    mtb.mtb_tune_reset()
    mtb.mtb_set_shape(4, 1100, 700, 3300, 6, {"pyramid_slots_pct": 150, "pyramid_tile_group": 2,
                                              "bitmaps_waves": 8, "coarse_levels": 2, "level1_from_level0": 1,
                                              "search_rows": [16] * 16, "search_lanes": [32] * 16})
    before = mtb.mtb_tuned_shape(4, 1100, 700, 3300, 6)
    path = str(tmp_path / "shapes.txt")
    mtb.mtb_tune_save(path)
    first = open(path).readline().split()
    assert first[:2] == ["mtb-tune", "3"] and first[2].startswith("gfx950") and first[3].startswith("hip-")
    mtb.mtb_tune_reset()
    assert mtb.mtb_tuned_shape(4, 1100, 700, 3300, 6) is None
    assert mtb.mtb_tune_load(path) == 1
    assert mtb.mtb_tuned_shape(4, 1100, 700, 3300, 6) == before
    # A file written on another platform is skipped whole.
    other = str(tmp_path / "other.txt")
    lines = open(path).read().splitlines()
    open(other, "w").write("\n".join(["mtb-tune 3 gfx942 hip-1"] + lines[1:]) + "\n")
    mtb.mtb_tune_reset()
    assert mtb.mtb_tune_load(other) == 0
    assert mtb.mtb_tuned_shape(4, 1100, 700, 3300, 6) is None
    mtb.mtb_tune_reset()


def test_tuned_batch_groups_keep_results(mtb):
    items = []
    for k, (w, h, L) in enumerate([(640, 480, 5), (900, 600, 6), (640, 480, 5), (900, 600, 6), (640, 480, 5)]):
        ref, mov, _ = synth.make_rect_pair(w, h, 20, 610 + k, (1 << (L - 1)) - 1)
        items.append((ref, mov, L))
    dev = [(torch.from_numpy(r).to(DEV), torch.from_numpy(m).to(DEV), L) for r, m, L in items]
    mtb.mtb_tune_reset()
    base = mtb.mtb_align_batch(dev)
    torch.cuda.synchronize()
    b_sh, b_er = base["shifts"].cpu().numpy(), base["errs"].cpu().numpy()
    assert mtb.mtb_tune_batch(dev) == 2
    assert mtb.mtb_tuned_shape(6, 640, 480, 1920, 5) is not None
    assert mtb.mtb_tuned_shape(4, 900, 600, 2700, 6) is not None
    got = mtb.mtb_align_batch(dev)
    torch.cuda.synchronize()
    assert np.array_equal(got["shifts"].cpu().numpy(), b_sh)
    assert np.array_equal(got["errs"].cpu().numpy(), b_er)
    want = np.array([oracle.align_pair(r, m, L)["shift"] for r, m, L in items], dtype=np.int32)
    assert np.array_equal(b_sh, want)
    mtb.mtb_tune_reset()
