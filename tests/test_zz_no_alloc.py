"""The allocation-free pair search (mtb_align_pair_scratch, search state in the
library's static device array) against mtb_align_pair with a workspace, through
the C ABI: calls in a row on the same device, each on a smaller pair with fewer
levels than the one before, and every output (shift, error, the nine errors
and the chosen shift of every level) must be identical; each pair is also
checked against the oracle."""

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


def _bitmaps(mtb, img, L):
    d = torch.from_numpy(img).to(DEV)
    pyr = mtb.mtb_build_pyramid(d, L)
    h, w = img.shape[:2]
    return mtb.mtb_bitmaps(pyr, w, h, L)


def test_scratch_search_equals_workspace_search(mtb):
    # Second call: a smaller input with fewer levels that still keeps its
    # search state in the static array; third: a pair small enough for the
    # one-workgroup search, which keeps none.
    cases = [(1024, 768, 7, 50, 3), (640, 480, 5, 12, 7), (300, 200, 4, 12, 9)]
    for w, h, L, t, seed in cases:
        ref, mov, _ = synth.make_rect_pair(w, h, 24, seed, t)
        bref, bmov = _bitmaps(mtb, ref, L), _bitmaps(mtb, mov, L)
        want = mtb.mtb_align_pair(bref, bmov, w, h, L, trace=True, level_shifts=True)
        shift = torch.full((2,), -99, dtype=torch.int32, device=DEV)
        err = torch.full((1,), -1, dtype=torch.int32, device=DEV)
        tr = torch.full((L, 9), -1, dtype=torch.int32, device=DEV)
        ls = torch.full((L, 2), -99, dtype=torch.int32, device=DEV)
        got = mtb.mtb_align_pair_scratch(bref, bmov, w, h, L, shift, err, tr, ls)
        torch.cuda.synchronize()
        for k in ("shift", "err", "trace", "level_shifts"):
            assert torch.equal(got[k], want[k]), (w, h, L, k)
        o = oracle.align_pair(ref, mov, L)
        assert tuple(shift.cpu().numpy()) == tuple(o["shift"]), (w, h, L)
        assert int(err.item()) == int(o["err"]), (w, h, L)
        assert np.array_equal(tr.cpu().numpy().astype(np.int64), o["trace"]), (w, h, L)
