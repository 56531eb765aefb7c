"""CPU oracle for MTB translational alignment -- test infrastructure only.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product path (the HIP library and its binding) never
does, and shares no code with it: the arithmetic lives in ``mtb_oracle.c``,
plain single-threaded C with one byte per pixel, following the paper's steps
in its order (see the comments there).  This module only marshals numpy arrays
into that library and, for stacks, runs independent images and pairs on a
thread pool.

Results use the paper's notation: level l of an image W x H is W>>l by H>>l;
a shift (dx, dy) is what must be applied to the moving image,
aligned[y][x] = mov[y - dy][x - dx].
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mtb_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

__all__ = [
    "quadrants",
    "align_quadrants",
    "apply_shift",
    "align_stack_chained",
    "build",
    "gray",
    "downsample",
    "histogram",
    "median",
    "bitmaps",
    "shift_error",
    "pyramid",
    "search",
    "align_pair",
    "align_stack",
    "max_levels",
]


def build(force: bool = True) -> str:
    """Compile liboracle.so next to its source (gcc, plain C11)."""
    global _lib
    if force or not os.path.exists(_LIB):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.run(
            ["gcc", "-std=c11", "-O2", "-Wall", "-Wextra", "-Werror", "-shared", "-fPIC",
             _SRC, "-o", tmp],
            check=True,
        )
        os.replace(tmp, _LIB)
        _lib = None
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    i32, i64 = ctypes.c_int32, ctypes.c_int64
    lib.oracle_level_offset.argtypes = [i32, i32, i32]
    lib.oracle_level_offset.restype = i64
    lib.oracle_gray.argtypes = [P, i32, i32, i64, P]
    lib.oracle_gray.restype = None
    lib.oracle_downsample.argtypes = [P, i32, i32, P]
    lib.oracle_downsample.restype = None
    lib.oracle_histogram.argtypes = [P, i64, P]
    lib.oracle_histogram.restype = None
    lib.oracle_median.argtypes = [P, i64]
    lib.oracle_median.restype = i32
    lib.oracle_bitmaps.argtypes = [P, i64, i32, i32, P, P]
    lib.oracle_bitmaps.restype = None
    lib.oracle_shift_error.argtypes = [P, P, P, P, i32, i32, i32, i32]
    lib.oracle_shift_error.restype = i64
    lib.oracle_pyramid.argtypes = [P, i32, i32, i64, i32, P, P, P]
    lib.oracle_pyramid.restype = None
    lib.oracle_pyramid_bitmaps.argtypes = [P, i32, i32, i32, P, i32, P, P]
    lib.oracle_pyramid_bitmaps.restype = None
    lib.oracle_search.argtypes = [P, P, P, P, i32, i32, i32, P, P, P, P]
    lib.oracle_search.restype = None
    lib.oracle_align_pair.argtypes = [P, P, i32, i32, i64, i32, i32, P, P, P, P]
    lib.oracle_align_pair.restype = i32
    lib.oracle_apply_shift.argtypes = [P, i32, i32, i64, i32, i32, i32, P, i64]
    lib.oracle_apply_shift.restype = None
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _rgb(img: np.ndarray):
    """(H, W, 3) uint8 image, or a (H, stride) byte view of one -> (array, W, H, stride)."""
    a = np.asarray(img)
    if a.dtype != np.uint8 or a.ndim != 3 or a.shape[2] != 3:
        raise ValueError("expected an (H, W, 3) uint8 image")
    if a.strides[2] != 1 or a.strides[1] != 3:
        a = np.ascontiguousarray(a)
    return a, a.shape[1], a.shape[0], a.strides[0]


def max_levels(width: int, height: int) -> int:
    """Largest L such that level L-1 is at least one pixel in each dimension."""
    L = 0
    while (width >> L) >= 1 and (height >> L) >= 1:
        L += 1
    return L


def gray(img: np.ndarray) -> np.ndarray:
    a, W, H, s = _rgb(img)
    out = np.empty((H, W), np.uint8)
    _load().oracle_gray(_ptr(a), W, H, s, _ptr(out))
    return out


def downsample(g: np.ndarray) -> np.ndarray:
    g = np.ascontiguousarray(g, dtype=np.uint8)
    H, W = g.shape
    out = np.empty((H >> 1, W >> 1), np.uint8)
    _load().oracle_downsample(_ptr(g), W, H, _ptr(out))
    return out


def histogram(g: np.ndarray) -> np.ndarray:
    g = np.ascontiguousarray(g, dtype=np.uint8)
    h = np.empty(256, np.uint32)
    _load().oracle_histogram(_ptr(g), g.size, _ptr(h))
    return h


def median(hist: np.ndarray, npix: int) -> int:
    h = np.ascontiguousarray(hist, dtype=np.uint32)
    return int(_load().oracle_median(_ptr(h), int(npix)))


def bitmaps(g: np.ndarray, m: int, exclude: int = 4):
    g = np.ascontiguousarray(g, dtype=np.uint8)
    t = np.empty_like(g)
    e = np.empty_like(g)
    _load().oracle_bitmaps(_ptr(g), g.size, int(m), int(exclude), _ptr(t), _ptr(e))
    return t, e


def shift_error(tr, er, tm, em, cx: int, cy: int) -> int:
    arrs = [np.ascontiguousarray(a, dtype=np.uint8) for a in (tr, er, tm, em)]
    H, W = arrs[0].shape
    for a in arrs:
        if a.shape != (H, W):
            raise ValueError("bitmaps must share one shape")
    return int(_load().oracle_shift_error(*(_ptr(a) for a in arrs), W, H, int(cx), int(cy)))


class Pyramid:
    """Gray levels, histograms, medians and bitmaps of one image (byte per pixel)."""

    def __init__(self, width, height, levels, flat_gray, hist, med, flat_t, flat_e):
        self.width, self.height, self.levels = width, height, levels
        self.flat_gray, self.hist, self.median = flat_gray, hist, med
        self.flat_t, self.flat_e = flat_t, flat_e

    def _level(self, flat, l):
        lib = _load()
        off = lib.oracle_level_offset(self.width, self.height, l)
        w, h = self.width >> l, self.height >> l
        return flat[off:off + w * h].reshape(h, w)

    def gray(self, l):
        return self._level(self.flat_gray, l)

    def tb(self, l):
        return self._level(self.flat_t, l)

    def eb(self, l):
        return self._level(self.flat_e, l)


def pyramid(img: np.ndarray, levels: int, exclude: int = 4) -> Pyramid:
    """Gray pyramid, per-level histograms and medians, and per-level bitmaps."""
    a, W, H, s = _rgb(img)
    if not 1 <= levels <= max_levels(W, H):
        raise ValueError("levels out of range")
    lib = _load()
    total = lib.oracle_level_offset(W, H, levels)
    g = np.empty(total, np.uint8)
    hist = np.empty((levels, 256), np.uint32)
    med = np.empty(levels, np.int32)
    lib.oracle_pyramid(_ptr(a), W, H, s, levels, _ptr(g), _ptr(hist), _ptr(med))
    t = np.empty(total, np.uint8)
    e = np.empty(total, np.uint8)
    lib.oracle_pyramid_bitmaps(_ptr(g), W, H, levels, _ptr(med), int(exclude), _ptr(t), _ptr(e))
    return Pyramid(W, H, levels, g, hist, med, t, e)


def search(ref: Pyramid, mov: Pyramid) -> dict:
    """Coarse-to-fine 9-candidate search of ``mov`` against ``ref``."""
    if (ref.width, ref.height, ref.levels) != (mov.width, mov.height, mov.levels):
        raise ValueError("pyramids differ in size or level count")
    L = ref.levels
    shift = np.zeros(2, np.int32)
    err = np.zeros(1, np.int64)
    trace = np.zeros((L, 9), np.int64)
    lvl = np.zeros((L, 2), np.int32)
    _load().oracle_search(_ptr(ref.flat_t), _ptr(ref.flat_e), _ptr(mov.flat_t), _ptr(mov.flat_e),
                          ref.width, ref.height, L, _ptr(shift), _ptr(err), _ptr(trace), _ptr(lvl))
    return {"shift": (int(shift[0]), int(shift[1])), "err": int(err[0]),
            "trace": trace, "level_shifts": lvl}


def align_pair(ref_img: np.ndarray, mov_img: np.ndarray, levels: int, exclude: int = 4) -> dict:
    """End-to-end alignment of one pair: pyramids and bitmaps of both, then the search."""
    pr = pyramid(ref_img, levels, exclude)
    pm = pyramid(mov_img, levels, exclude)
    out = search(pr, pm)
    out["ref"], out["mov"] = pr, pm
    return out


def align_stack(images, levels: int, ref_index: int | None = None, exclude: int = 4,
                threads: int = 1, keep: bool = False) -> dict:
    """Align every image of a stack against the reference (middle image by default).

    Each image's pyramid and bitmaps are built once; the N-1 searches all use
    the reference's.  ``threads`` > 1 runs independent images, then independent
    pairs, concurrently (the C calls release the GIL).  The reference reports
    shift (0, 0) and error 0.
    """
    n = len(images)
    if n < 1:
        raise ValueError("empty stack")
    ref = n // 2 if ref_index is None or ref_index < 0 else int(ref_index)
    if not 0 <= ref < n:
        raise ValueError("ref_index out of range")
    shape = np.asarray(images[0]).shape
    for im in images:
        if np.asarray(im).shape != shape:
            raise ValueError("all images of a stack must share one size")
    with ThreadPoolExecutor(max_workers=max(1, threads)) as ex:
        pyrs = list(ex.map(lambda im: pyramid(im, levels, exclude), images))
        others = [k for k in range(n) if k != ref]
        res = dict(zip(others, ex.map(lambda k: search(pyrs[ref], pyrs[k]), others)))
    shifts = np.zeros((n, 2), np.int32)
    errs = np.zeros(n, np.int64)
    for k, r in res.items():
        shifts[k] = r["shift"]
        errs[k] = r["err"]
    out = {"shifts": shifts, "errs": errs, "ref_index": ref, "pairs": res}
    if keep:
        out["pyramids"] = pyrs
    return out


def align_stack_chained(images, levels: int, ref_index: int | None = None, exclude: int = 4,
                        threads: int = 1) -> dict:
    """Chained stack alignment: image k against its neighbour towards the reference
    (k + 1 below it, k - 1 above), the pairwise shifts summed along the chain
    (translations compose by addition; Section III-A compares consecutive
    exposures, Section III-B aligns a stack pairwise).

    Returns ``shifts`` (summed, against the reference), ``errs`` and ``pairs``
    (pairwise results, keyed by the moving image).
    """
    n = len(images)
    if n < 1:
        raise ValueError("empty stack")
    ref = n // 2 if ref_index is None or ref_index < 0 else int(ref_index)
    if not 0 <= ref < n:
        raise ValueError("ref_index out of range")
    with ThreadPoolExecutor(max_workers=max(1, threads)) as ex:
        pyrs = list(ex.map(lambda im: pyramid(im, levels, exclude), images))
        others = [k for k in range(n) if k != ref]
        nb = {k: (k + 1 if k < ref else k - 1) for k in others}
        res = dict(zip(others, ex.map(lambda k: search(pyrs[nb[k]], pyrs[k]), others)))
    shifts = np.zeros((n, 2), np.int64)
    errs = np.zeros(n, np.int64)
    for k in list(range(ref - 1, -1, -1)) + list(range(ref + 1, n)):
        shifts[k] = np.array(res[k]["shift"]) + shifts[nb[k]]
        errs[k] = res[k]["err"]
    return {"shifts": shifts.astype(np.int32), "errs": errs, "ref_index": ref, "pairs": res}


def apply_shift(img: np.ndarray, dx: int, dy: int, fill: int = 0) -> np.ndarray:
    """out[y][x] = img[y - dy][x - dx]; outside the image: zeros (fill 0) or the
    nearest edge pixel (fill 1).  Returns a packed (H, W, 3) image."""
    a, W, H, s = _rgb(img)
    out = np.empty((H, W, 3), np.uint8)
    _load().oracle_apply_shift(_ptr(a), W, H, s, int(dx), int(dy), int(fill), _ptr(out), 3 * W)
    return out


def quadrants(img: np.ndarray):
    """The four quadrants (top-left, top-right, bottom-left, bottom-right) of an
    (H, W, 3) image, split at column W // 2 and row H // 2."""
    a = np.asarray(img)
    H, W = a.shape[:2]
    w0, h0 = W // 2, H // 2
    return [a[:h0, :w0], a[:h0, w0:], a[h0:, :w0], a[h0:, w0:]]


def align_quadrants(ref_img: np.ndarray, mov_img: np.ndarray, levels: int, exclude: int = 4,
                    tolerance: int = 1) -> dict:
    """Align each quadrant pair on its own (Section II, after Ward: quadrants that
    disagree reveal a rotation).  The flag is raised when two quadrants' shifts
    differ by more than `tolerance` along either axis."""
    res = [align_pair(np.ascontiguousarray(r), np.ascontiguousarray(m), levels, exclude)
           for r, m in zip(quadrants(ref_img), quadrants(mov_img))]
    shifts = np.array([r["shift"] for r in res], np.int32)
    errs = np.array([r["err"] for r in res], np.int64)
    spread = (shifts.max(axis=0) - shifts.min(axis=0)).max()
    return {"shifts": shifts, "errs": errs, "flag": int(spread > tolerance)}
