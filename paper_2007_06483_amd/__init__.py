"""Python binding of libmtb: MTB translational alignment on MI355X (gfx950).

Thin ctypes marshalling over the C ABI declared in include/mtb.h; the
functions keep the C names.  Every step of the computation runs in the HIP
kernels of libmtb.so; PyTorch only provides device memory (CUDA/HIP tensors)
and the current stream.  There is no CPU fallback: if libmtb.so is missing,
or no gfx950 device is usable, the calls raise.

Build the library in-tree first (``python -m paper_2007_06483_amd._build`` or
``__graft_entry__.build()``).
"""

from __future__ import annotations

import ctypes
import os

import torch

__all__ = [
    "MTBError",
    "Layout",
    "MTB_MAX_LEVELS",
    "MTB_MAX_STACK",
    "library_path",
    "lib",
    "mtb_status_string",
    "mtb_max_levels",
    "mtb_get_layout",
    "mtb_pyramid_bytes",
    "mtb_bitmaps_bytes",
    "mtb_pair_workspace_bytes",
    "mtb_stack_workspace_bytes",
    "mtb_build_pyramid",
    "mtb_bitmaps",
    "mtb_align_pair",
    "mtb_align_pair_scratch",
    "mtb_align_stack",
    "mtb_align_stack_chained",
    "mtb_align_stack_bytemaps",
    "mtb_stack_bytemaps_workspace_bytes",
    "mtb_apply_shifts",
    "mtb_stage_rgb",
    "mtb_tune_stack",
    "mtb_set_shape",
    "mtb_tuned_shape",
    "mtb_tune_reset",
    "mtb_tune_save",
    "mtb_tune_load",
    "mtb_tune_batch",
    "mtb_test_fail_launch",
    "mtb_test_last_pyramid",
    "mtb_stack_image_buffers",
    "mtb_level1_from_level0",
    "mtb_quadrant_workspace_bytes",
    "mtb_align_quadrants",
    "MTB_FILL_ZERO",
    "MTB_FILL_EDGE",
    "mtb_batch_workspace_bytes",
    "mtb_align_batch",
    "mtb_batch_stacks_workspace_bytes",
    "mtb_align_batch_stacks",
    "mtb_profile_begin",
    "mtb_profile_end",
    "mtb_profile_pause",
    "mtb_probe_stream",
]

MTB_MAX_LEVELS = 16
MTB_MAX_STACK = 32
MTB_MAX_BATCH = 4096
MTB_FILL_ZERO = 0
MTB_FILL_EDGE = 1

MTB_OK = 0
STATUS_NAMES = {0: "MTB_OK", 1: "MTB_ERR_INVALID_ARG", 2: "MTB_ERR_WORKSPACE",
                3: "MTB_ERR_DEVICE", 4: "MTB_ERR_UNSUPPORTED"}

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libmtb.so")
_lib = None


class MTBError(RuntimeError):
    """A libmtb call returned a status other than MTB_OK."""

    def __init__(self, func: str, status: int):
        self.status = int(status)
        super().__init__(f"{func} failed: {STATUS_NAMES.get(self.status, self.status)}")


class _CLayout(ctypes.Structure):
    _fields_ = [
        ("width", ctypes.c_int32),
        ("height", ctypes.c_int32),
        ("levels", ctypes.c_int32),
        ("level_width", ctypes.c_int32 * MTB_MAX_LEVELS),
        ("level_height", ctypes.c_int32 * MTB_MAX_LEVELS),
        ("words_per_row", ctypes.c_int32 * MTB_MAX_LEVELS),
        ("gray_offset", ctypes.c_int64 * MTB_MAX_LEVELS),
        ("gray_pitch", ctypes.c_int64 * MTB_MAX_LEVELS),
        ("hist_offset", ctypes.c_int64),
        ("pyramid_bytes", ctypes.c_int64),
        ("tb_offset", ctypes.c_int64 * MTB_MAX_LEVELS),
        ("eb_offset", ctypes.c_int64 * MTB_MAX_LEVELS),
        ("median_offset", ctypes.c_int64),
        ("bitmaps_bytes", ctypes.c_int64),
    ]


class _BatchStack(ctypes.Structure):
    _fields_ = [("d_rgb", ctypes.POINTER(ctypes.c_void_p)), ("n", ctypes.c_int32), ("ref_index", ctypes.c_int32),
                ("row_stride", ctypes.c_int64), ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("levels", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class _BatchItem(ctypes.Structure):
    _fields_ = [("d_ref_rgb", ctypes.c_void_p), ("d_mov_rgb", ctypes.c_void_p),
                ("row_stride", ctypes.c_int64), ("width", ctypes.c_int32),
                ("height", ctypes.c_int32), ("levels", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class _KernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double)]


class _LaunchShape(ctypes.Structure):
    _fields_ = [("pyramid_slots_pct", ctypes.c_int32), ("pyramid_tile_group", ctypes.c_int32),
                ("bitmaps_blocks_pct", ctypes.c_int32), ("bitmaps_waves", ctypes.c_int32),
                ("coarse_levels", ctypes.c_int32), ("small_search", ctypes.c_int32),
                ("level1_from_level0", ctypes.c_int32),
                ("search_rows", ctypes.c_int32 * MTB_MAX_LEVELS),
                ("search_lanes", ctypes.c_int32 * MTB_MAX_LEVELS), ("step_ms", ctypes.c_float),
                ("default_ms", ctypes.c_float)]


_SHAPE_DEFAULTS = {"pyramid_slots_pct": 100, "pyramid_tile_group": 1, "bitmaps_blocks_pct": 100,
                   "bitmaps_waves": 4, "coarse_levels": -1, "small_search": -1, "level1_from_level0": -1}


def _shape_dict(c: _LaunchShape) -> dict:
    d = {k: int(getattr(c, k)) for k in _SHAPE_DEFAULTS}
    d.update({"search_rows": list(c.search_rows), "search_lanes": list(c.search_lanes),
              "step_ms": float(c.step_ms), "default_ms": float(c.default_ms)})
    return d


def _shape_struct(d: dict) -> _LaunchShape:
    rows = list(d.get("search_rows", [])) + [0] * MTB_MAX_LEVELS
    lanes = list(d.get("search_lanes", [])) + [0] * MTB_MAX_LEVELS
    v = {k: int(d.get(k, dv)) for k, dv in _SHAPE_DEFAULTS.items()}
    return _LaunchShape(v["pyramid_slots_pct"], v["pyramid_tile_group"], v["bitmaps_blocks_pct"],
                        v["bitmaps_waves"], v["coarse_levels"], v["small_search"], v["level1_from_level0"],
                        (ctypes.c_int32 * MTB_MAX_LEVELS)(*rows[:MTB_MAX_LEVELS]),
                        (ctypes.c_int32 * MTB_MAX_LEVELS)(*lanes[:MTB_MAX_LEVELS]), 0.0, 0.0)


class Layout:
    """Offsets (bytes) of every level inside the pyramid and bitmaps buffers."""

    def __init__(self, c: _CLayout):
        L = c.levels
        self.width, self.height, self.levels = c.width, c.height, L
        self.level_width = list(c.level_width[:L])
        self.level_height = list(c.level_height[:L])
        self.words_per_row = list(c.words_per_row[:L])
        self.gray_offset = list(c.gray_offset[:L])
        self.gray_pitch = list(c.gray_pitch[:L])
        self.hist_offset = c.hist_offset
        self.pyramid_bytes = c.pyramid_bytes
        self.tb_offset = list(c.tb_offset[:L])
        self.eb_offset = list(c.eb_offset[:L])
        self.median_offset = c.median_offset
        self.bitmaps_bytes = c.bitmaps_bytes


def library_path() -> str:
    return _LIB_PATH


def lib():
    """The loaded libmtb.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"libmtb.so is not built ({_LIB_PATH}); run paper_2007_06483_amd._build.build()")
    L = ctypes.CDLL(_LIB_PATH)
    P, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    L.mtb_status_string.argtypes = [ctypes.c_int]
    L.mtb_status_string.restype = ctypes.c_char_p
    L.mtb_max_levels.argtypes = [i32, i32]
    L.mtb_max_levels.restype = i32
    L.mtb_get_layout.argtypes = [i32, i32, i32, ctypes.POINTER(_CLayout)]
    L.mtb_get_layout.restype = ctypes.c_int
    for f in ("mtb_pyramid_bytes", "mtb_bitmaps_bytes"):
        getattr(L, f).argtypes = [i32, i32, i32]
        getattr(L, f).restype = sz
    L.mtb_pair_workspace_bytes.argtypes = [i32]
    L.mtb_pair_workspace_bytes.restype = sz
    L.mtb_stack_workspace_bytes.argtypes = [i32, i32, i32, i32]
    L.mtb_stack_workspace_bytes.restype = sz
    L.mtb_build_pyramid.argtypes = [P, i32, i32, i64, i32, P, sz, P]
    L.mtb_build_pyramid.restype = ctypes.c_int
    L.mtb_bitmaps.argtypes = [P, i32, i32, i32, i32, P, sz, P]
    L.mtb_bitmaps.restype = ctypes.c_int
    L.mtb_align_pair.argtypes = [P, P, i32, i32, i32, P, sz, P, P, P, P, P]
    L.mtb_align_pair_scratch.argtypes = [P, P, i32, i32, i32, P, P, P, P, P]
    L.mtb_align_pair_scratch.restype = ctypes.c_int
    L.mtb_align_pair.restype = ctypes.c_int
    L.mtb_align_stack.argtypes = [ctypes.POINTER(P), i32, i32, i32, i64, i32, i32, i32, P, sz, P, P, P, P]
    L.mtb_align_stack.restype = ctypes.c_int
    L.mtb_align_stack_chained.argtypes = L.mtb_align_stack.argtypes
    L.mtb_align_stack_chained.restype = ctypes.c_int
    L.mtb_align_stack_bytemaps.argtypes = L.mtb_align_stack.argtypes
    L.mtb_align_stack_bytemaps.restype = ctypes.c_int
    L.mtb_stack_bytemaps_workspace_bytes.argtypes = [i32, i32, i32, i32]
    L.mtb_stack_bytemaps_workspace_bytes.restype = sz
    L.mtb_quadrant_workspace_bytes.argtypes = [i32, i32, i64, i32]
    L.mtb_quadrant_workspace_bytes.restype = sz
    L.mtb_align_quadrants.argtypes = [P, P, i32, i32, i64, i32, i32, i32, P, sz, P, P, P, P]
    L.mtb_align_quadrants.restype = ctypes.c_int
    L.mtb_apply_shifts.argtypes = [ctypes.POINTER(P), i32, i32, i32, i64, P, i32, ctypes.POINTER(P), i64, P]
    L.mtb_apply_shifts.restype = ctypes.c_int
    L.mtb_tune_stack.argtypes = [ctypes.POINTER(P), i32, i32, i32, i64, i32, i32, i32, P, sz, P, P, P,
                                 ctypes.POINTER(_LaunchShape)]
    L.mtb_tune_stack.restype = ctypes.c_int
    L.mtb_set_shape.argtypes = [i32, i32, i32, i64, i32, ctypes.POINTER(_LaunchShape)]
    L.mtb_set_shape.restype = ctypes.c_int
    L.mtb_tuned_shape.argtypes = [i32, i32, i32, i64, i32, ctypes.POINTER(_LaunchShape)]
    L.mtb_tuned_shape.restype = ctypes.c_int
    L.mtb_tune_reset.argtypes = []
    L.mtb_tune_reset.restype = None
    L.mtb_tune_save.argtypes = [ctypes.c_char_p]
    L.mtb_tune_save.restype = ctypes.c_int
    L.mtb_tune_load.argtypes = [ctypes.c_char_p, ctypes.POINTER(i32)]
    L.mtb_tune_load.restype = ctypes.c_int
    L.mtb_test_fail_launch.argtypes = [i32]
    L.mtb_test_fail_launch.restype = ctypes.c_int
    L.mtb_test_last_pyramid.argtypes = [ctypes.POINTER(i32), ctypes.POINTER(i32)]
    L.mtb_test_last_pyramid.restype = ctypes.c_int
    L.mtb_stack_image_buffers.argtypes = [P, i32, i32, i32, i32, ctypes.POINTER(P), ctypes.POINTER(P)]
    L.mtb_stack_image_buffers.restype = ctypes.c_int
    L.mtb_level1_from_level0.argtypes = [i32, i32, i32, i64, i32]
    L.mtb_level1_from_level0.restype = i32
    L.mtb_stage_rgb.argtypes = [P, i64, i32, i32, P, i64, P]
    L.mtb_stage_rgb.restype = ctypes.c_int
    L.mtb_batch_workspace_bytes.argtypes = [ctypes.POINTER(_BatchItem), i32]
    L.mtb_batch_workspace_bytes.restype = sz
    L.mtb_align_batch.argtypes = [ctypes.POINTER(_BatchItem), i32, i32, P, sz, P, P, P]
    L.mtb_batch_stacks_workspace_bytes.argtypes = [ctypes.POINTER(_BatchStack), i32]
    L.mtb_batch_stacks_workspace_bytes.restype = sz
    L.mtb_align_batch_stacks.argtypes = [ctypes.POINTER(_BatchStack), i32, i32, P, sz, P, P, P]
    L.mtb_align_batch_stacks.restype = ctypes.c_int
    L.mtb_probe_stream.argtypes = [P, sz, P, sz, P]
    L.mtb_probe_stream.restype = ctypes.c_int
    L.mtb_tune_batch.argtypes = [ctypes.POINTER(_BatchItem), i32, i32, P, sz, P, P, P, ctypes.POINTER(i32)]
    L.mtb_tune_batch.restype = ctypes.c_int
    L.mtb_align_batch.restype = ctypes.c_int
    L.mtb_profile_pause.argtypes = [i32]
    L.mtb_profile_pause.restype = ctypes.c_int
    L.mtb_profile_begin.argtypes = [ctypes.c_char_p]
    L.mtb_profile_begin.restype = ctypes.c_int
    L.mtb_profile_end.argtypes = [ctypes.POINTER(_KernelTime), i32, ctypes.POINTER(i32)]
    L.mtb_profile_end.restype = ctypes.c_int
    _lib = L
    return L


def _check(func: str, status: int):
    if status != MTB_OK:
        raise MTBError(func, status)


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    if isinstance(stream, torch.cuda.Stream):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _device_u8(t: torch.Tensor, what: str):
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.uint8:
        raise TypeError(f"{what} must be a uint8 tensor on a GPU")


def _rgb_geometry(img: torch.Tensor):
    """(H, W, 3) uint8 device tensor with packed pixels -> (W, H, row_stride_bytes)."""
    _device_u8(img, "image")
    if img.dim() != 3 or img.shape[2] != 3 or img.stride(2) != 1 or img.stride(1) != 3:
        raise ValueError("image must be (H, W, 3) with interleaved R,G,B bytes")
    return int(img.shape[1]), int(img.shape[0]), int(img.stride(0))


def mtb_status_string(status: int) -> str:
    return lib().mtb_status_string(int(status)).decode()


def mtb_max_levels(width: int, height: int) -> int:
    return int(lib().mtb_max_levels(width, height))


def mtb_get_layout(width: int, height: int, levels: int) -> Layout:
    c = _CLayout()
    _check("mtb_get_layout", lib().mtb_get_layout(width, height, levels, ctypes.byref(c)))
    return Layout(c)


def mtb_pyramid_bytes(width: int, height: int, levels: int) -> int:
    return int(lib().mtb_pyramid_bytes(width, height, levels))


def mtb_bitmaps_bytes(width: int, height: int, levels: int) -> int:
    return int(lib().mtb_bitmaps_bytes(width, height, levels))


def mtb_pair_workspace_bytes(levels: int) -> int:
    return int(lib().mtb_pair_workspace_bytes(levels))


def mtb_stack_workspace_bytes(n: int, width: int, height: int, levels: int) -> int:
    return int(lib().mtb_stack_workspace_bytes(n, width, height, levels))


def _buffer(nbytes: int, device, out=None) -> torch.Tensor:
    if out is None:
        return torch.empty(nbytes, dtype=torch.uint8, device=device)
    _device_u8(out, "output buffer")
    return out


def mtb_build_pyramid(rgb: torch.Tensor, levels: int, pyramid: torch.Tensor | None = None,
                      stream=None) -> torch.Tensor:
    """Gray pyramid and histograms of one (H, W, 3) RGB image; returns the pyramid buffer."""
    W, H, stride = _rgb_geometry(rgb)
    need = mtb_pyramid_bytes(W, H, levels)
    pyramid = _buffer(max(need, 1), rgb.device, pyramid)
    _check("mtb_build_pyramid",
           lib().mtb_build_pyramid(_ptr(rgb), W, H, stride, levels, _ptr(pyramid),
                                   pyramid.numel(), _stream(stream)))
    return pyramid


def mtb_bitmaps(pyramid: torch.Tensor, width: int, height: int, levels: int, exclude_range: int = 4,
                bitmaps: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Medians and packed threshold/exclusion bitmaps of a pyramid; returns the bitmaps buffer."""
    _device_u8(pyramid, "pyramid")
    need = mtb_bitmaps_bytes(width, height, levels)
    bitmaps = _buffer(max(need, 1), pyramid.device, bitmaps)
    _check("mtb_bitmaps",
           lib().mtb_bitmaps(_ptr(pyramid), width, height, levels, exclude_range, _ptr(bitmaps),
                             bitmaps.numel(), _stream(stream)))
    return bitmaps


def mtb_align_pair(bm_ref: torch.Tensor, bm_mov: torch.Tensor, width: int, height: int,
                   levels: int, workspace: torch.Tensor | None = None, trace: bool = False,
                   level_shifts: bool = False, shift=None, err=None, stream=None) -> dict:
    """Coarse-to-fine search of the moving bitmaps against the reference's.

    Returns device tensors ``shift`` int32[2] (dx, dy), ``err`` int32[1] (the uint32
    level-0 count, below 2^31) and optionally ``trace`` int32[levels][9] and
    ``level_shifts`` int32[levels][2].
    """
    _device_u8(bm_ref, "bm_ref")
    _device_u8(bm_mov, "bm_mov")
    dev = bm_ref.device
    workspace = _buffer(max(mtb_pair_workspace_bytes(levels), 1), dev, workspace)
    if shift is None:
        shift = torch.empty(2, dtype=torch.int32, device=dev)
    if err is None:
        err = torch.empty(1, dtype=torch.int32, device=dev)
    tr = torch.empty((levels, 9), dtype=torch.int32, device=dev) if trace else None
    ls = torch.empty((levels, 2), dtype=torch.int32, device=dev) if level_shifts else None
    _check("mtb_align_pair",
           lib().mtb_align_pair(_ptr(bm_ref), _ptr(bm_mov), width, height, levels, _ptr(workspace),
                                workspace.numel(), _ptr(shift), _ptr(err), _ptr(tr), _ptr(ls),
                                _stream(stream)))
    return {"shift": shift, "err": err, "trace": tr, "level_shifts": ls}


def mtb_align_pair_scratch(bm_ref: torch.Tensor, bm_mov: torch.Tensor, width: int, height: int,
                           levels: int, shift: torch.Tensor, err: torch.Tensor, trace: torch.Tensor | None = None,
                           level_shifts: torch.Tensor | None = None, stream=None) -> dict:
    """mtb_align_pair with the search state in the library's static device array
    (no workspace; the caller passes every output, so nothing is allocated here)."""
    _device_u8(bm_ref, "bm_ref")
    _device_u8(bm_mov, "bm_mov")
    for t, n, what in ((shift, 2, "shift"), (err, 1, "err"), (trace, 9 * levels, "trace"),
                       (level_shifts, 2 * levels, "level_shifts")):
        if t is not None and (t.dtype != torch.int32 or not t.is_contiguous() or t.numel() < n):
            raise ValueError(f"{what}: a contiguous int32 tensor of at least {n} elements")
    _check("mtb_align_pair_scratch",
           lib().mtb_align_pair_scratch(_ptr(bm_ref), _ptr(bm_mov), width, height, levels, _ptr(shift), _ptr(err),
                                        _ptr(trace), _ptr(level_shifts), _stream(stream)))
    return {"shift": shift, "err": err, "trace": trace, "level_shifts": level_shifts}


def mtb_align_stack_chained(images, levels: int, exclude_range: int = 4, ref_index: int = -1,
                            workspace: torch.Tensor | None = None, trace: bool = False, shifts=None,
                            errs=None, stream=None) -> dict:
    """Chained stack: each image against its neighbour towards the reference, shifts summed.

    Same arguments and results as mtb_align_stack; ``errs`` and ``trace`` are pairwise.
    """
    return mtb_align_stack(images, levels, exclude_range, ref_index, workspace, trace, shifts, errs,
                           stream, _entry="mtb_align_stack_chained")


def mtb_stack_bytemaps_workspace_bytes(n: int, width: int, height: int, levels: int) -> int:
    return int(lib().mtb_stack_bytemaps_workspace_bytes(n, width, height, levels))


def mtb_align_stack_bytemaps(images, levels: int, exclude_range: int = 4, ref_index: int = -1,
                             workspace: torch.Tensor | None = None, trace: bool = False, shifts=None,
                             errs=None, stream=None) -> dict:
    """The stack through byte maps (255/0 per pixel), the paper's representation; same results."""
    return mtb_align_stack(images, levels, exclude_range, ref_index, workspace, trace, shifts, errs,
                           stream, _entry="mtb_align_stack_bytemaps")


def mtb_align_stack(images, levels: int, exclude_range: int = 4, ref_index: int = -1,
                    workspace: torch.Tensor | None = None, trace: bool = False, shifts=None,
                    errs=None, stream=None, _entry: str = "mtb_align_stack") -> dict:
    """Align every (H, W, 3) image of a stack against the reference (n // 2 by default).

    Returns device tensors ``shifts`` int32[n][2], ``errs`` int32[n] (the uint32
    counts, which stay below 2^31) and, with trace=True, ``trace`` int32[n][levels][9].
    """
    n = len(images)
    if not 1 <= n <= MTB_MAX_STACK:
        raise ValueError(f"a stack holds 1..{MTB_MAX_STACK} images")
    W, H, stride = _rgb_geometry(images[0])
    for im in images:
        if _rgb_geometry(im) != (W, H, stride) or im.device != images[0].device:
            raise ValueError("all images of a stack must share size, stride and device")
    dev = images[0].device
    need = (mtb_stack_bytemaps_workspace_bytes if _entry == "mtb_align_stack_bytemaps"
            else mtb_stack_workspace_bytes)(n, W, H, levels)
    workspace = _buffer(max(need, 1), dev, workspace)
    if shifts is None:
        shifts = torch.empty((n, 2), dtype=torch.int32, device=dev)
    if errs is None:
        errs = torch.empty(n, dtype=torch.int32, device=dev)
    tr = torch.empty((n, levels, 9), dtype=torch.int32, device=dev) if trace else None
    ptrs = (ctypes.c_void_p * n)(*[im.data_ptr() for im in images])
    _check(_entry,
           getattr(lib(), _entry)(ptrs, n, W, H, stride, levels, exclude_range, ref_index,
                                  _ptr(workspace), workspace.numel(), _ptr(shifts), _ptr(errs),
                                  _ptr(tr), _stream(stream)))
    return {"shifts": shifts, "errs": errs, "trace": tr, "workspace": workspace}


def mtb_tune_stack(images, levels: int, exclude_range: int = 4, ref_index: int = -1,
                   workspace: torch.Tensor | None = None, shifts=None, errs=None, stream=None) -> dict:
    """Tune and store the launch shape of mtb_align_stack for this stack (see mtb.h).

    Returns the chosen shape as a dict (with step_ms and default_ms); the
    stack's shifts and errors are left in ``shifts`` / ``errs`` if given.
    """
    n = len(images)
    if not 1 <= n <= MTB_MAX_STACK:
        raise ValueError(f"a stack holds 1..{MTB_MAX_STACK} images")
    W, H, stride = _rgb_geometry(images[0])
    for im in images:
        if _rgb_geometry(im) != (W, H, stride) or im.device != images[0].device:
            raise ValueError("all images of a stack must share size, stride and device")
    dev = images[0].device
    workspace = _buffer(max(mtb_stack_workspace_bytes(n, W, H, levels), 1), dev, workspace)
    if shifts is None:
        shifts = torch.empty((n, 2), dtype=torch.int32, device=dev)
    if errs is None:
        errs = torch.empty(n, dtype=torch.int32, device=dev)
    ptrs = (ctypes.c_void_p * n)(*[im.data_ptr() for im in images])
    out = _LaunchShape()
    _check("mtb_tune_stack",
           lib().mtb_tune_stack(ptrs, n, W, H, stride, levels, exclude_range, ref_index, _ptr(workspace),
                                workspace.numel(), _ptr(shifts), _ptr(errs), _stream(stream), ctypes.byref(out)))
    return _shape_dict(out)


def mtb_set_shape(n: int, width: int, height: int, row_stride: int, levels: int, shape: dict) -> None:
    c = _shape_struct(shape)
    _check("mtb_set_shape", lib().mtb_set_shape(n, width, height, row_stride, levels, ctypes.byref(c)))


def mtb_tuned_shape(n: int, width: int, height: int, row_stride: int, levels: int):
    """The stored shape for the key, or None."""
    c = _LaunchShape()
    if lib().mtb_tuned_shape(n, width, height, row_stride, levels, ctypes.byref(c)) != MTB_OK:
        return None
    return _shape_dict(c)


def mtb_tune_reset() -> None:
    lib().mtb_tune_reset()


def mtb_tune_save(path: str) -> None:
    """Write every stored launch shape (with the device architecture and HIP version) to ``path``."""
    _check("mtb_tune_save", lib().mtb_tune_save(os.fsencode(path)))


def mtb_tune_load(path: str) -> int:
    """Store the shapes of a file written by mtb_tune_save on this architecture and HIP
    version; returns how many were stored (0 for a file from another platform)."""
    n = ctypes.c_int32(0)
    _check("mtb_tune_load", lib().mtb_tune_load(os.fsencode(path), ctypes.byref(n)))
    return int(n.value)


def mtb_test_fail_launch(after: int) -> None:
    """Make this thread's launch after `after` successful ones fail, once (tests only)."""
    _check("mtb_test_fail_launch", lib().mtb_test_fail_launch(int(after)))


def mtb_test_last_pyramid() -> tuple:
    """(workgroups, merged) of this thread's last k_pyramid launch (tests only)."""
    blocks, merged = ctypes.c_int32(0), ctypes.c_int32(0)
    _check("mtb_test_last_pyramid", lib().mtb_test_last_pyramid(ctypes.byref(blocks), ctypes.byref(merged)))
    return int(blocks.value), bool(merged.value)


def mtb_stack_image_buffers(workspace: torch.Tensor, n: int, width: int, height: int, levels: int):
    """Byte offsets into ``workspace`` of each image's (pyramid, bitmaps) buffer after mtb_align_stack."""
    _device_u8(workspace, "workspace")
    pyr = (ctypes.c_void_p * n)()
    bms = (ctypes.c_void_p * n)()
    _check("mtb_stack_image_buffers",
           lib().mtb_stack_image_buffers(_ptr(workspace), n, width, height, levels, pyr, bms))
    base = workspace.data_ptr()
    return [(int(pyr[i]) - base, int(bms[i]) - base) for i in range(n)]


def mtb_level1_from_level0(n: int, width: int, height: int, row_stride: int, levels: int) -> bool:
    """Whether the alignment calls for n images of this size form level 1's bitmaps
    from level 0's gray (and leave level 1's gray out of the workspace)."""
    r = lib().mtb_level1_from_level0(n, width, height, row_stride, levels)
    if r < 0:
        raise MTBError("mtb_level1_from_level0", 1)  # MTB_ERR_INVALID_ARG
    return bool(r)


def mtb_apply_shifts(images, shifts: torch.Tensor, fill: int = MTB_FILL_ZERO, out=None,
                     stream=None) -> list:
    """Translate every (H, W, 3) image by its row of ``shifts`` (device int32[n][2]).

    Returns the output images (new packed tensors unless ``out`` gives them).
    """
    n = len(images)
    if not 1 <= n <= MTB_MAX_STACK:
        raise ValueError(f"a stack holds 1..{MTB_MAX_STACK} images")
    W, H, stride = _rgb_geometry(images[0])
    for im in images:
        if _rgb_geometry(im) != (W, H, stride):
            raise ValueError("all images must share size and stride")
    if (not isinstance(shifts, torch.Tensor) or not shifts.is_cuda or shifts.dtype != torch.int32
            or tuple(shifts.shape) != (n, 2) or not shifts.is_contiguous()):
        raise ValueError("shifts must be a contiguous int32 device tensor of shape (n, 2)")
    if out is None:
        out = [torch.empty((H, W, 3), dtype=torch.uint8, device=images[0].device) for _ in range(n)]
    ostride = None
    for o in out:
        ow, oh, os_ = _rgb_geometry(o)
        if (ow, oh) != (W, H) or (ostride is not None and os_ != ostride):
            raise ValueError("outputs must match the inputs' size and share a stride")
        ostride = os_
    ins = (ctypes.c_void_p * n)(*[im.data_ptr() for im in images])
    outs = (ctypes.c_void_p * n)(*[o.data_ptr() for o in out])
    _check("mtb_apply_shifts",
           lib().mtb_apply_shifts(ins, n, W, H, stride, _ptr(shifts), int(fill), outs, ostride,
                                  _stream(stream)))
    return out


def mtb_stage_rgb(host: torch.Tensor, dst: torch.Tensor, stream=None) -> torch.Tensor:
    """Enqueue the copy of a host (H, W, 3) RGB image (a view; pinned for an
    asynchronous copy) into the device image ``dst`` of the same size."""
    if (not isinstance(host, torch.Tensor) or host.device.type != "cpu" or host.dtype != torch.uint8
            or host.dim() != 3 or host.shape[2] != 3 or host.stride(2) != 1 or host.stride(1) != 3):
        raise ValueError("host must be a CPU uint8 (H, W, 3) view with interleaved R,G,B bytes")
    W, H, dstride = _rgb_geometry(dst)
    if (int(host.shape[1]), int(host.shape[0])) != (W, H):
        raise ValueError("host and dst must have the same size")
    _check("mtb_stage_rgb",
           lib().mtb_stage_rgb(host.data_ptr(), int(host.stride(0)), W, H, dst.data_ptr(), dstride,
                               _stream(stream)))
    return dst


def mtb_quadrant_workspace_bytes(width: int, height: int, row_stride: int, levels: int) -> int:
    return int(lib().mtb_quadrant_workspace_bytes(width, height, row_stride, levels))


def mtb_align_quadrants(ref: torch.Tensor, mov: torch.Tensor, levels: int, exclude_range: int = 4,
                        tolerance: int = 1, workspace: torch.Tensor | None = None, stream=None) -> dict:
    """Align the four quadrant pairs of (ref, mov); flag a suspected rotation.

    Returns device tensors ``shifts`` int32[4][2], ``errs`` int32[4], ``flag`` int32[1].
    """
    W, H, stride = _rgb_geometry(ref)
    if _rgb_geometry(mov) != (W, H, stride):
        raise ValueError("both images must share size and stride")
    dev = ref.device
    need = mtb_quadrant_workspace_bytes(W, H, stride, levels)
    workspace = _buffer(max(need, 1), dev, workspace)
    shifts = torch.empty((4, 2), dtype=torch.int32, device=dev)
    errs = torch.empty(4, dtype=torch.int32, device=dev)
    flag = torch.empty(1, dtype=torch.int32, device=dev)
    _check("mtb_align_quadrants",
           lib().mtb_align_quadrants(_ptr(ref), _ptr(mov), W, H, stride, levels, exclude_range, tolerance,
                                     _ptr(workspace), workspace.numel(), _ptr(shifts), _ptr(errs),
                                     _ptr(flag), _stream(stream)))
    return {"shifts": shifts, "errs": errs, "flag": flag}


def _batch_items(pairs):
    """[(ref, mov, levels), ...] of (H, W, 3) device images -> ctypes item array."""
    n = len(pairs)
    if not 1 <= n <= MTB_MAX_BATCH:
        raise ValueError(f"a batch holds 1..{MTB_MAX_BATCH} items")
    items = (_BatchItem * n)()
    for i, (ref, mov, levels) in enumerate(pairs):
        geo = _rgb_geometry(ref)
        if _rgb_geometry(mov) != geo or mov.device != ref.device:
            raise ValueError("the two images of an item must share size, stride and device")
        W, H, stride = geo
        items[i] = _BatchItem(ref.data_ptr(), mov.data_ptr(), stride, W, H, int(levels), 0)
    return items


def mtb_batch_workspace_bytes(pairs) -> int:
    """Workspace bytes for mtb_align_batch over [(ref, mov, levels), ...]."""
    items = _batch_items(pairs)
    return int(lib().mtb_batch_workspace_bytes(items, len(pairs)))


def mtb_align_batch(pairs, exclude_range: int = 4, workspace: torch.Tensor | None = None,
                    shifts=None, errs=None, stream=None) -> dict:
    """Align every (ref, mov, levels) item of a batch; sizes may differ between items.

    Returns device tensors ``shifts`` int32[n][2] and ``errs`` int32[n].
    """
    items = _batch_items(pairs)
    n = len(pairs)
    dev = pairs[0][0].device
    need = int(lib().mtb_batch_workspace_bytes(items, n))
    workspace = _buffer(max(need, 1), dev, workspace)
    if shifts is None:
        shifts = torch.empty((n, 2), dtype=torch.int32, device=dev)
    if errs is None:
        errs = torch.empty(n, dtype=torch.int32, device=dev)
    _check("mtb_align_batch",
           lib().mtb_align_batch(items, n, exclude_range, _ptr(workspace), workspace.numel(),
                                 _ptr(shifts), _ptr(errs), _stream(stream)))
    return {"shifts": shifts, "errs": errs, "workspace": workspace}


def _batch_stacks(stacks):
    """[(images, levels[, ref_index]), ...] -> (ctypes item array, pointer arrays to keep alive,
    first output row of each stack, rows)."""
    n = len(stacks)
    if not 1 <= n <= MTB_MAX_BATCH:
        raise ValueError(f"a batch holds 1..{MTB_MAX_BATCH} items")
    items = (_BatchStack * n)()
    keep, starts, rows = [], [], 0
    for i, st in enumerate(stacks):
        images, levels = st[0], st[1]
        ref = -1 if len(st) < 3 or st[2] is None else int(st[2])
        if not 1 <= len(images) <= MTB_MAX_STACK:
            raise ValueError(f"a stack holds 1..{MTB_MAX_STACK} images")
        geo = _rgb_geometry(images[0])
        for im in images[1:]:
            if _rgb_geometry(im) != geo or im.device != images[0].device:
                raise ValueError("the images of a stack must share size, stride and device")
        W, H, stride = geo
        ptrs = (ctypes.c_void_p * len(images))(*[im.data_ptr() for im in images])
        keep.append(ptrs)
        items[i] = _BatchStack(ctypes.cast(ptrs, ctypes.POINTER(ctypes.c_void_p)), len(images), ref, stride, W, H,
                               int(levels), 0)
        starts.append(rows)
        rows += len(images)
    return items, keep, starts, rows


def mtb_batch_stacks_workspace_bytes(stacks) -> int:
    """Workspace bytes for mtb_align_batch_stacks over [(images, levels[, ref_index]), ...]."""
    items, _keep, _, _ = _batch_stacks(stacks)
    return int(lib().mtb_batch_stacks_workspace_bytes(items, len(stacks)))


def mtb_align_batch_stacks(stacks, exclude_range: int = 4, workspace: torch.Tensor | None = None,
                           shifts=None, errs=None, stream=None) -> dict:
    """Align every exposure stack (images, levels[, ref_index]) of a batch; sizes may differ
    between stacks.  Returns device tensors ``shifts`` int32[rows][2] and ``errs`` int32[rows]
    (one row per image, stacks one after another) and ``starts``, each stack's first row."""
    items, _keep, starts, rows = _batch_stacks(stacks)
    dev = stacks[0][0][0].device
    need = int(lib().mtb_batch_stacks_workspace_bytes(items, len(stacks)))
    workspace = _buffer(max(need, 1), dev, workspace)
    if shifts is None:
        shifts = torch.empty((rows, 2), dtype=torch.int32, device=dev)
    if errs is None:
        errs = torch.empty(rows, dtype=torch.int32, device=dev)
    _check("mtb_align_batch_stacks",
           lib().mtb_align_batch_stacks(items, len(stacks), exclude_range, _ptr(workspace), workspace.numel(),
                                        _ptr(shifts), _ptr(errs), _stream(stream)))
    return {"shifts": shifts, "errs": errs, "starts": starts, "workspace": workspace}


def mtb_tune_batch(pairs, exclude_range: int = 4, workspace: torch.Tensor | None = None,
                   shifts=None, errs=None, stream=None) -> int:
    """Tune and store the launch shape of every group key of a batch (see mtb_align_batch);
    returns the number of keys tuned.  shifts/errs (if given) receive the batch's results."""
    items = _batch_items(pairs)
    n = len(pairs)
    dev = pairs[0][0].device
    need = int(lib().mtb_batch_workspace_bytes(items, n))
    workspace = _buffer(max(need, 1), dev, workspace)
    if shifts is None:
        shifts = torch.empty((n, 2), dtype=torch.int32, device=dev)
    if errs is None:
        errs = torch.empty(n, dtype=torch.int32, device=dev)
    tuned = ctypes.c_int32(0)
    _check("mtb_tune_batch",
           lib().mtb_tune_batch(items, n, exclude_range, _ptr(workspace), workspace.numel(), _ptr(shifts),
                                _ptr(errs), _stream(stream), ctypes.byref(tuned)))
    return int(tuned.value)


def mtb_probe_stream(src: torch.Tensor, read_bytes: int, dst: torch.Tensor | None, write_bytes: int,
                     stream=None) -> None:
    """One launch of the streaming yardstick kernel (reads read_bytes of src, writes write_bytes of dst)."""
    _device_u8(src, "src")
    if read_bytes > src.numel() or (write_bytes > 0 and (dst is None or write_bytes > dst.numel())):
        raise ValueError("buffers smaller than the bytes to stream")
    _check("mtb_probe_stream", lib().mtb_probe_stream(_ptr(src), read_bytes, _ptr(dst), write_bytes,
                                                      _stream(stream)))


def mtb_profile_begin(kernel_name: str | None = None) -> None:
    """Start timing the library's kernel launches on this thread (optionally one kernel name)."""
    _check("mtb_profile_begin", lib().mtb_profile_begin(None if kernel_name is None else kernel_name.encode()))


def mtb_profile_pause(paused: bool) -> None:
    """Stop (True) or resume (False) bracketing launches while profiling is on."""
    _check("mtb_profile_pause", lib().mtb_profile_pause(1 if paused else 0))


def mtb_profile_end(capacity: int = 64) -> dict:
    """Stop timing; returns {kernel name: (launches, total milliseconds)}."""
    out = (_KernelTime * capacity)()
    count = ctypes.c_int32(0)
    _check("mtb_profile_end", lib().mtb_profile_end(out, capacity, ctypes.byref(count)))
    return {out[i].name.decode(): (int(out[i].launches), float(out[i].total_ms)) for i in range(count.value)}
