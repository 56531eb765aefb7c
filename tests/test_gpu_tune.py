"""Launch shapes never change results: the tuner's choice and explicit shapes
(pyramid and bitmap grids from a quarter to four rounds, every fine level's
rows per stream from 4 to 64) give bit-identical shifts, errors and traces,
equal to the oracle's."""

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
    assert all(r == 0 or (r % 4 == 0 and 4 <= r <= 64) for r in shape["search_rows"])
    assert shape["step_ms"] > 0 and shape["default_ms"] > 0
    assert shape["step_ms"] <= shape["default_ms"]
    stored = mtb.mtb_tuned_shape(5, 900, 640, 2700, L)
    assert stored is not None
    assert {k: stored[k] for k in ("pyramid_slots_pct", "bitmaps_blocks_pct", "search_rows")} == \
        {k: shape[k] for k in ("pyramid_slots_pct", "bitmaps_blocks_pct", "search_rows")}
    after = _run(mtb, d, L)
    for a, b in zip(before, after):
        assert np.array_equal(a, b)
    want = oracle.align_stack(imgs, L, threads=4)
    assert np.array_equal(after[0], want["shifts"])
    assert np.array_equal(after[1].astype(np.int64), want["errs"])


@pytest.mark.parametrize("pyr,bm", [(25, 25), (50, 100), (200, 50), (400, 100)])
def test_explicit_shapes_give_identical_results(mtb, pyr, bm):
    imgs, d = _stack(4, 1100, 700, 62, 30)
    L = 6
    mtb.mtb_tune_reset()
    ref = _run(mtb, d, L)
    for rows in (4, 8, 28, 64):
        mtb.mtb_set_shape(4, 1100, 700, 3300, L, {"pyramid_slots_pct": pyr, "bitmaps_blocks_pct": bm,
                                                  "search_rows": [rows] * 16})
        got = _run(mtb, d, L)
        for a, b in zip(ref, got):
            assert np.array_equal(a, b), (pyr, bm, rows)
    mtb.mtb_tune_reset()
