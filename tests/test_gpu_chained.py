"""Chained stack alignment (mtb_align_stack_chained) against the oracle, bit-exact:
summed shifts, pairwise errors and pairwise per-level traces."""

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
    return m


def _check(mtb, imgs, L, ref_index=None):
    want = oracle.align_stack_chained(imgs, L, ref_index=ref_index, threads=4)
    d = [torch.from_numpy(np.ascontiguousarray(im)).to(DEV) for im in imgs]
    got = mtb.mtb_align_stack_chained(d, L, ref_index=-1 if ref_index is None else ref_index, trace=True)
    torch.cuda.synchronize()
    assert np.array_equal(got["shifts"].cpu().numpy(), want["shifts"])
    assert np.array_equal(got["errs"].cpu().numpy().astype(np.int64), want["errs"])
    tr = got["trace"].cpu().numpy().astype(np.int64)
    for k, r in want["pairs"].items():
        assert np.array_equal(tr[k], r["trace"]), k
    assert not tr[want["ref_index"]].any()
    return got, want


@pytest.mark.parametrize("n", [1, 2, 3, 5, 7])
def test_chained_blob_stacks(mtb, n):
    imgs, _, _ = synth.make_stack(640, 480, n, 80, 60 + n, 30, sat_frac=0.05)
    _check(mtb, imgs, 6)


@pytest.mark.parametrize("ref", [0, 2, 4])
def test_chained_reference_positions(mtb, ref):
    rng = np.random.default_rng(70 + ref)
    rad = synth.rect_field(300, 200, 25, rng)
    imgs = [synth.translate(synth.expose(rad, float(e)), int(rng.integers(-7, 8)), int(rng.integers(-7, 8)))
            for e in (-2, -1, 0, 1, 2)]
    _check(mtb, imgs, 5, ref_index=ref)


@pytest.mark.timeout(900)
def test_chained_full_size_stack(mtb):
    w = synth.workload("stack7_6000x4000")
    (imgs, _, ref), = w.stacks
    _check(mtb, imgs, w.levels, ref_index=ref)
