"""Applying shifts to a stack (mtb_apply_shifts) against the oracle, bit-exact.

Covers both fill readings, shifts larger than the image, odd widths, padded
and unaligned rows (the byte path) and the shifts straight from
mtb_align_stack on the 7 x 6000x4000 stack.
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


def _dev(img, extra=0, offset=0):
    """Device (H, W, 3) view with rows 3W + extra bytes apart, starting offset bytes in."""
    h, w, _ = img.shape
    stride = 3 * w + extra
    buf = torch.full((offset + stride * h + 16,), 7, dtype=torch.uint8, device=DEV)
    rows = buf[offset:offset + stride * h].view(h, stride)
    rows[:, :3 * w] = torch.from_numpy(np.ascontiguousarray(img).reshape(h, 3 * w)).to(DEV)
    return torch.as_strided(buf, (h, w, 3), (stride, 3, 1), offset)


def _check(mtb, imgs, shifts, fill, extra=0, offset=0, out_extra=0):
    d = [_dev(im, extra, offset) for im in imgs]
    sh = torch.tensor(shifts, dtype=torch.int32, device=DEV)
    h, w, _ = imgs[0].shape
    outs = [_dev(np.zeros_like(im), out_extra) for im in imgs]
    mtb.mtb_apply_shifts(d, sh, fill, out=outs)
    torch.cuda.synchronize()
    for im, o, (dx, dy) in zip(imgs, outs, shifts):
        want = oracle.apply_shift(im, dx, dy, fill)
        assert np.array_equal(o.cpu().numpy(), want), (im.shape, dx, dy, fill)


@pytest.mark.parametrize("fill", [0, 1])
@pytest.mark.parametrize("h,w", [(1, 1), (3, 5), (37, 61), (64, 96), (130, 301), (256, 1000)])
def test_apply_shifts_matches_oracle(mtb, fill, h, w):
    rng = np.random.default_rng(h * 1000 + w)
    imgs = [rng.integers(0, 256, (h, w, 3), dtype=np.uint8) for _ in range(5)]
    shifts = [(0, 0), (1, -1), (-w - 2, 3), (w // 2 + 1, -(h // 3) - 1), (-7, h + 4)]
    _check(mtb, imgs, shifts, fill)


@pytest.mark.parametrize("extra,offset,out_extra", [(1, 0, 0), (4, 4, 16), (5, 3, 1), (0, 16, 7)])
def test_apply_shifts_strides_and_alignment(mtb, extra, offset, out_extra):
    rng = np.random.default_rng(extra * 100 + offset)
    imgs = [rng.integers(0, 256, (45, 83, 3), dtype=np.uint8) for _ in range(3)]
    for fill in (0, 1):
        _check(mtb, imgs, [(3, 2), (-11, -5), (0, 0)], fill, extra, offset, out_extra)


def test_apply_shifts_leaves_row_padding_untouched(mtb):
    img = np.random.default_rng(5).integers(0, 256, (20, 30, 3), dtype=np.uint8)
    out = _dev(np.zeros_like(img), 6)
    sh = torch.tensor([[4, -3]], dtype=torch.int32, device=DEV)
    mtb.mtb_apply_shifts([_dev(img)], sh, 0, out=[out])
    torch.cuda.synchronize()
    base = out.as_strided((20 * 96,), (1,), out.storage_offset()).cpu().numpy().reshape(20, 96)
    assert (base[:, 90:] == 7).all()


@pytest.mark.timeout(900)
def test_apply_stack_shifts_full_size(mtb):
    w = synth.workload("stack7_6000x4000")
    (imgs, _, ref), = w.stacks
    d = [torch.from_numpy(im).to(DEV) for im in imgs]
    got = mtb.mtb_align_stack(d, w.levels, ref_index=ref)
    for fill in (0, 1):
        outs = mtb.mtb_apply_shifts(d, got["shifts"], fill)
        torch.cuda.synchronize()
        shifts = got["shifts"].cpu().numpy()
        for k in (0, 3, 6):
            want = oracle.apply_shift(imgs[k], int(shifts[k][0]), int(shifts[k][1]), fill)
            assert np.array_equal(outs[k].cpu().numpy(), want), (k, fill)
