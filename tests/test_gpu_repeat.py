"""Repeated runs of the two protocols that exchange data between workgroups
of one launch without device-wide fences:

* the pyramid's histogram merge through per-XCD copies and tile tickets
  (one 2048x1536 image: 192 workgroups for its 192 tiles, the merge path);
* the search's tickets (the last workgroup of the level-0 launch sums every
  pair's counters and writes the outputs), on the 7-image 6000x4000 stack.

Each is run back to back many times on the same stream and every result is
compared with the oracle (and with the first run); the test stops at the
first difference.
"""

import numpy as np
import pytest

import oracle
import synth
from mtb_decode import histograms

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

DEV = "cuda:0"
REPEATS = 200


@pytest.fixture(scope="module")
def mtb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2007_06483_amd as m

    m.lib()
    return m


def test_histogram_merge_repeated(mtb):
    w, h, L = 2048, 1536, 6
    imgs, _, _ = synth.make_stack(w, h, 1, 60, 4242, 0, sat_frac=0.02)
    want = oracle.pyramid(imgs[0], L, 4).hist
    d = torch.from_numpy(imgs[0]).to(DEV)
    lay = mtb.mtb_get_layout(w, h, L)
    pyr = torch.empty(mtb.mtb_pyramid_bytes(w, h, L), dtype=torch.uint8, device=DEV)
    for k in range(REPEATS):
        mtb.mtb_build_pyramid(d, L, pyramid=pyr)
        if k == 0:
            blocks, merged = mtb.mtb_test_last_pyramid()
            assert merged, f"{blocks} workgroups did not take the merge path"
        got = histograms(pyr.cpu().numpy(), lay)
        assert np.array_equal(got, want), f"histograms differ from the oracle at run {k}"


@pytest.mark.timeout(900)
def test_stack_tickets_repeated(mtb):
    wl = synth.workload("stack7_6000x4000")
    (imgs, _, ref), = wl.stacks
    L = wl.levels
    want = oracle.align_stack(imgs, L, ref_index=ref)
    d = [torch.from_numpy(im).to(DEV) for im in imgs]
    first = mtb.mtb_align_stack(d, L, ref_index=ref, trace=True)
    torch.cuda.synchronize()
    f_shifts, f_errs, f_trace = first["shifts"].clone(), first["errs"].clone(), first["trace"].clone()
    assert np.array_equal(f_shifts.cpu().numpy(), want["shifts"])
    assert np.array_equal(f_errs.cpu().numpy().astype(np.int64), want["errs"])
    tr = f_trace.cpu().numpy().astype(np.int64)
    for k, r in want["pairs"].items():
        assert np.array_equal(tr[k], r["trace"]), f"trace of image {k}"
    ws, shifts, errs = first["workspace"], torch.empty_like(f_shifts), torch.empty_like(f_errs)
    for k in range(REPEATS):
        shifts.fill_(-99)
        errs.fill_(-1)
        got = mtb.mtb_align_stack(d, L, ref_index=ref, workspace=ws, trace=True, shifts=shifts, errs=errs)
        torch.cuda.synchronize()
        assert torch.equal(shifts, f_shifts), f"shifts differ at run {k}"
        assert torch.equal(errs, f_errs), f"errors differ at run {k}"
        assert torch.equal(got["trace"], f_trace), f"trace differs at run {k}"


@pytest.mark.timeout(600)
def test_alternating_stacks_share_one_workspace(mtb):
    """Two different stacks of one size alternate through the same workspace:
    every call must give its own stack's results (shifts, errors, all nine
    errors of every level), whatever the previous call left in the buffers
    and in the caches of any XCD."""
    w, h, L, n = 3000, 2000, 7, 5
    ref = n // 2
    want, dev = [], []
    for seed in (11, 12):
        imgs, _, _ = synth.make_stack(w, h, n, 200, seed, 40, sat_frac=0.03)
        want.append(oracle.align_stack(imgs, L, ref_index=ref))
        dev.append([torch.from_numpy(im).to(DEV) for im in imgs])
    assert not np.array_equal(want[0]["shifts"], want[1]["shifts"])
    ws = torch.empty(mtb.mtb_stack_workspace_bytes(n, w, h, L), dtype=torch.uint8, device=DEV)
    out = torch.empty((n, 2), dtype=torch.int32, device=DEV)
    errs = torch.empty(n, dtype=torch.int32, device=DEV)
    for k in range(60):
        s = k % 2
        out.fill_(-99)
        got = mtb.mtb_align_stack(dev[s], L, ref_index=ref, workspace=ws, trace=True, shifts=out, errs=errs)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), want[s]["shifts"]), f"shifts of stack {s} at run {k}"
        assert np.array_equal(errs.cpu().numpy().astype(np.int64), want[s]["errs"]), f"errors at run {k}"
        tr = got["trace"].cpu().numpy().astype(np.int64)
        for i, r in want[s]["pairs"].items():
            assert np.array_equal(tr[i], r["trace"]), f"trace of image {i} of stack {s} at run {k}"
