"""The byte-map path (the paper's 255/0 representation) gives the same shifts,
errors and traces as the oracle and as the packed path, bit-exact."""

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


def _check(mtb, imgs, L, ref_index=None, exclude=4):
    want = oracle.align_stack(imgs, L, ref_index=ref_index, exclude=exclude, threads=4)
    d = [torch.from_numpy(np.ascontiguousarray(im)).to(DEV) for im in imgs]
    ri = -1 if ref_index is None else ref_index
    got = mtb.mtb_align_stack_bytemaps(d, L, exclude_range=exclude, ref_index=ri, trace=True)
    packed = mtb.mtb_align_stack(d, L, exclude_range=exclude, ref_index=ri, trace=True)
    torch.cuda.synchronize()
    assert np.array_equal(got["shifts"].cpu().numpy(), want["shifts"])
    assert np.array_equal(got["errs"].cpu().numpy().astype(np.int64), want["errs"])
    tr = got["trace"].cpu().numpy().astype(np.int64)
    for k, r in want["pairs"].items():
        assert np.array_equal(tr[k], r["trace"]), k
    assert torch.equal(got["trace"], packed["trace"])


@pytest.mark.parametrize("w,h,L", [(320, 240, 5), (333, 211, 6), (97, 61, 3), (1, 40, 1), (700, 5, 2)])
def test_bytemaps_rect_pairs(mtb, w, h, L):
    ref, mov, _ = synth.make_rect_pair(w, h, max(4, w * h // 4000), w + h, (1 << (L - 1)) - 1)
    _check(mtb, [ref, mov], L, ref_index=0)


@pytest.mark.parametrize("exclude", [0, 4, 200])
def test_bytemaps_stacks(mtb, exclude):
    imgs, _, _ = synth.make_stack(640, 480, 5, 80, 90 + exclude, 25, sat_frac=0.05)
    _check(mtb, imgs, 6, exclude=exclude)


@pytest.mark.timeout(900)
def test_bytemaps_full_size_stack(mtb):
    w = synth.workload("stack7_6000x4000")
    (imgs, _, ref), = w.stacks
    _check(mtb, imgs, w.levels, ref_index=ref)
