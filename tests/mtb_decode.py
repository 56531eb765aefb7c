"""Host-side decoding of libmtb's device buffers into plain numpy arrays.

Only layout arithmetic (offsets from mtb_get_layout, bit unpacking); no part
of the alignment method.  Used by the parity tests to compare every
intermediate with the oracle.
"""

import numpy as np


def gray_levels(buf: np.ndarray, layout):
    out = []
    for l in range(layout.levels):
        w, h = layout.level_width[l], layout.level_height[l]
        off, pitch = layout.gray_offset[l], layout.gray_pitch[l]
        out.append(buf[off:off + pitch * h].reshape(h, pitch)[:, :w])
    return out


def histograms(buf: np.ndarray, layout) -> np.ndarray:
    off = layout.hist_offset
    return buf[off:off + 1024 * layout.levels].view(np.uint32).reshape(layout.levels, 256)


def medians(bm: np.ndarray, layout) -> np.ndarray:
    off = layout.median_offset
    return bm[off:off + 4 * layout.levels].view(np.int32)


def _plane(bm, off, w, h, wpr):
    words = bm[off:off + 8 * wpr * h].view(np.uint64).reshape(h, wpr)
    bits = np.unpackbits(words.view(np.uint8), bitorder="little").reshape(h, wpr * 64)
    return bits[:, :w], bits[:, w:]


def bitmaps(bm: np.ndarray, layout):
    """Per level (T, E, T_pad_bits, E_pad_bits) as 0/1 uint8 arrays."""
    out = []
    for l in range(layout.levels):
        w, h, wpr = layout.level_width[l], layout.level_height[l], layout.words_per_row[l]
        t, tp = _plane(bm, layout.tb_offset[l], w, h, wpr)
        e, ep = _plane(bm, layout.eb_offset[l], w, h, wpr)
        out.append((t, e, tp, ep))
    return out


def stack_workspace(mtb, ws, n: int, layout):
    """Split an mtb_align_stack workspace (a device tensor) into per-image
    (pyramid, bitmaps) byte arrays, at the places mtb_stack_image_buffers names."""
    host = ws.cpu().numpy()
    offs = mtb.mtb_stack_image_buffers(ws, n, layout.width, layout.height, layout.levels)
    P, B = layout.pyramid_bytes, layout.bitmaps_bytes
    pyr = [host[p:p + P] for p, _ in offs]
    bms = [host[b:b + B] for _, b in offs]
    return pyr, bms
