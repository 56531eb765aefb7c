"""Batched alignment of pairs of uneven sizes (mtb_align_batch) against the oracle.

Every item's shift and level-0 error must equal the oracle's pairwise result
for that item alone, whatever else shares the batch, and a HIP-graph capture
of the call must reproduce the eager results on every replay.  Integer
method: tolerance zero.
"""

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


def _to_dev(img, extra=0):
    """Device (H, W, 3) view of img; rows 3W + 3*extra bytes apart."""
    h, w, _ = img.shape
    buf = torch.zeros((h, w + extra, 3), dtype=torch.uint8, device=DEV)
    buf[:, :w] = torch.from_numpy(np.ascontiguousarray(img)).to(DEV)
    return buf[:, :w]


def _expected(items):
    want = [oracle.align_pair(ref, mov, L) for ref, mov, L in items]
    return (np.array([w["shift"] for w in want], dtype=np.int32),
            np.array([w["err"] for w in want], dtype=np.int64))


def _check(mtb, items, extras=None):
    extras = extras or [0] * len(items)
    dev = [(_to_dev(r, x), _to_dev(m, x), L) for (r, m, L), x in zip(items, extras)]
    got = mtb.mtb_align_batch(dev)
    torch.cuda.synchronize()
    shifts, errs = _expected(items)
    assert np.array_equal(got["shifts"].cpu().numpy(), shifts)
    assert np.array_equal(got["errs"].cpu().numpy().astype(np.int64), errs)
    return got, dev


def _rect_items(specs, seed0):
    items = []
    for k, (w, h, L) in enumerate(specs):
        ref, mov, _ = synth.make_rect_pair(w, h, max(8, w * h // 4000), seed0 + k, (1 << (L - 1)) - 1)
        items.append((ref, mov, L))
    return items


def test_batch_of_uneven_sizes(mtb):
    specs = [(160, 120, 4), (321, 243, 5), (640, 480, 5), (97, 61, 3), (160, 120, 4),
             (640, 480, 5), (321, 243, 5), (33, 17, 2), (160, 120, 4), (1100, 90, 6)]
    items = _rect_items(specs, 700)
    # Row padding differs between items of one size, so they form separate groups.
    _check(mtb, items, extras=[0, 1, 0, 5, 3, 0, 0, 0, 0, 2])


def test_batch_larger_than_one_group(mtb):
    # 18 items of one size: groups of 16 and 2; results must not depend on the split.
    items = _rect_items([(96, 64, 3)] * 18, 900)
    _check(mtb, items)


def test_batch_item_alone_equals_item_in_batch(mtb):
    items = _rect_items([(200, 150, 4), (256, 256, 5), (200, 150, 4)], 950)
    got, _ = _check(mtb, items)
    for k, it in enumerate(items):
        alone, _ = _check(mtb, [it])
        assert torch.equal(alone["shifts"][0], got["shifts"][k])
        assert torch.equal(alone["errs"][0], got["errs"][k])


def test_batch_graph_replay(mtb):
    items = _rect_items([(320, 240, 5), (128, 96, 4), (320, 240, 5), (257, 131, 4)], 970)
    dev = [(_to_dev(r), _to_dev(m), L) for r, m, L in items]
    eager = mtb.mtb_align_batch(dev)
    torch.cuda.synchronize()
    ref_shifts, ref_errs = eager["shifts"].clone(), eager["errs"].clone()
    ws = torch.empty_like(eager["workspace"])
    shifts = torch.empty_like(ref_shifts)
    errs = torch.empty_like(ref_errs)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # warm-up on the capture stream
        mtb.mtb_align_batch(dev, workspace=ws, shifts=shifts, errs=errs)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        mtb.mtb_align_batch(dev, workspace=ws, shifts=shifts, errs=errs)
    other = _rect_items([(200, 100, 4)], 990)
    other_dev = [(_to_dev(r), _to_dev(m), L) for r, m, L in other]
    for rep in range(3):
        shifts.fill_(-99)
        errs.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(shifts, ref_shifts), f"replay {rep}"
        assert torch.equal(errs, ref_errs), f"replay {rep}"
        # Eager work of the program between replays.
        mtb.mtb_align_batch(other_dev)
        torch.cuda.synchronize()


@pytest.mark.timeout(900)
def test_batch64_uneven_full_size(mtb):
    """The 64-pair uneven batch at full size: every item against the oracle."""
    import concurrent.futures

    batch = synth.make_batch(64, 4)
    dev = [(_to_dev(r), _to_dev(m), L) for r, m, _, L in batch]
    got = mtb.mtb_align_batch(dev)
    torch.cuda.synchronize()
    shifts = got["shifts"].cpu().numpy()
    errs = got["errs"].cpu().numpy().astype(np.int64)
    del dev

    def one(k):
        ref, mov, _, L = batch[k]
        w = oracle.align_pair(ref, mov, L)
        return w["shift"], w["err"]

    with concurrent.futures.ThreadPoolExecutor(max_workers=8) as ex:
        want = list(ex.map(one, range(len(batch))))
    for k, (shift, err) in enumerate(want):
        assert tuple(shifts[k]) == shift, k
        assert errs[k] == err, k


# ---------------------------------------------------------------- stacks as items


def _stack_specs():
    # (images, width, height, levels, reference or None for n // 2, extra row pixels): uneven
    # sizes, several stacks of one size sharing a launch set, single-image and two-image
    # stacks, a reference away from the middle, padded rows, and nine 4-image stacks of one
    # size (36 images: more than one launch set holds).
    specs = [(3, 640, 480, 5, None, 0), (5, 400, 300, 4, 0, 0), (2, 640, 480, 5, 1, 0), (1, 200, 150, 3, None, 0),
             (4, 900, 600, 6, None, 5), (3, 640, 480, 5, 2, 0)]
    specs += [(4, 320, 240, 4, None, 0)] * 9
    return specs


def test_stack_batch_matches_oracle_and_single_stacks(mtb):
    stacks, dev = [], []
    for k, (n, w, h, L, ref, extra) in enumerate(_stack_specs()):
        imgs, _, _ = synth.make_stack(w, h, n, max(8, w * h // 6000), 700 + k, min(w, h) // 8, sat_frac=0.05)
        stacks.append((imgs, L, ref))
        dev.append(([_to_dev(im, extra) for im in imgs], L, ref))
    got = mtb.mtb_align_batch_stacks(dev)
    torch.cuda.synchronize()
    g_sh, g_er = got["shifts"].cpu().numpy(), got["errs"].cpu().numpy().astype(np.int64)
    assert got["starts"][1] == 3 and len(g_sh) == sum(s[0] for s in _stack_specs())
    for (imgs, L, ref), (d, _, _), r0 in zip(stacks, dev, got["starts"]):
        n = len(imgs)
        want = oracle.align_stack(imgs, L, ref_index=ref, threads=4)
        assert np.array_equal(g_sh[r0:r0 + n], want["shifts"]), (n, L, ref)
        assert np.array_equal(g_er[r0:r0 + n], want["errs"]), (n, L, ref)
        alone = mtb.mtb_align_stack(d, L, ref_index=-1 if ref is None else ref)
        torch.cuda.synchronize()
        assert np.array_equal(alone["shifts"].cpu().numpy(), g_sh[r0:r0 + n])


def test_stack_batch_of_pairs_equals_pair_batch(mtb):
    # Two-image stacks with the reference first are the pair batch's items.
    items = _rect_items([(640, 480, 5), (321, 243, 5), (640, 480, 5)], 930)
    pairs = [(_to_dev(r), _to_dev(m), L) for r, m, L in items]
    by_pairs = mtb.mtb_align_batch(pairs)
    by_stacks = mtb.mtb_align_batch_stacks([([r, m], L, 0) for r, m, L in pairs])
    torch.cuda.synchronize()
    sh = by_stacks["shifts"].cpu().numpy().reshape(3, 2, 2)
    er = by_stacks["errs"].cpu().numpy().reshape(3, 2)
    assert np.array_equal(sh[:, 0], np.zeros((3, 2), np.int32)) and np.array_equal(er[:, 0], np.zeros(3))
    assert np.array_equal(sh[:, 1], by_pairs["shifts"].cpu().numpy())
    assert np.array_equal(er[:, 1], by_pairs["errs"].cpu().numpy())


def test_stack_batch_graph_replay(mtb):
    # The stacked batch (its output clearing included) captured once and
    # replayed: every replay reproduces the eager rows, with eager work of
    # the program between replays.
    dev = []
    for k, (n, w, h, L) in enumerate([(3, 320, 240, 5), (2, 128, 96, 4), (4, 320, 240, 5), (1, 64, 48, 3)]):
        imgs, _, _ = synth.make_stack(w, h, n, 12, 980 + k, min(w, h) // 8)
        dev.append(([_to_dev(im) for im in imgs], L, None))
    eager = mtb.mtb_align_batch_stacks(dev)
    torch.cuda.synchronize()
    ref_shifts, ref_errs = eager["shifts"].clone(), eager["errs"].clone()
    ws = torch.empty_like(eager["workspace"])
    shifts = torch.empty_like(ref_shifts)
    errs = torch.empty_like(ref_errs)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # warm-up on the capture stream
        mtb.mtb_align_batch_stacks(dev, workspace=ws, shifts=shifts, errs=errs)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        mtb.mtb_align_batch_stacks(dev, workspace=ws, shifts=shifts, errs=errs)
    other = _rect_items([(200, 100, 4)], 995)
    other_dev = [(_to_dev(r), _to_dev(m), L) for r, m, L in other]
    for rep in range(3):
        shifts.fill_(-99)
        errs.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(shifts, ref_shifts), f"replay {rep}"
        assert torch.equal(errs, ref_errs), f"replay {rep}"
        mtb.mtb_align_batch(other_dev)
        torch.cuda.synchronize()
