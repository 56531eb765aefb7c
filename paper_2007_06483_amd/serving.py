"""Served alignment: a request loop with continuous batching on one GPU.

Exposure stacks arrive over time.  A request is admitted as soon as an
execution slot (a HIP stream) is free and its workspace fits in the device
memory set aside for serving (admission by HBM footprint); requests that
arrive while others run are admitted as slots and memory free up, and the
stacks in flight overlap on the device.  Each admitted stack is one
``mtb_align_stack`` call on its slot's stream with a workspace carved out of
the serving pool; its pyramids and bitmaps stay on the device.  Latency is
completion minus arrival.

Requests are device-staged (their images already in device memory) or
host-staged (their images in host memory, pinned for asynchronous copies):
a host-staged request's footprint also holds device copies of its images,
which mtb_stage_rgb fills on the slot's stream before the alignment, so its
latency includes the host-to-device transfer.

The loop is host logic only: every step of the alignment runs in libmtb's
kernels.  The executor is a parameter so that the admission and retirement
logic can be exercised without a GPU.
"""

from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable


@dataclasses.dataclass
class Request:
    """One alignment request: a stack of same-size images (device tensors)."""

    rid: int
    arrival: float          # seconds after the start of the run
    images: list
    levels: int
    ref_index: int = -1
    exclude_range: int = 4
    workspace_bytes: int = 0
    megapixels: float = 0.0


@dataclasses.dataclass
class Result:
    rid: int
    arrival: float
    admitted: float
    completed: float
    shifts: object = None
    errs: object = None

    @property
    def latency(self) -> float:
        return self.completed - self.arrival


class FootprintPool:
    """First-fit allocator of byte ranges in a fixed region (alignment 256).

    Host-side bookkeeping only: it hands out offsets into one device buffer.
    """

    ALIGN = 256

    def __init__(self, capacity: int):
        if capacity <= 0:
            raise ValueError("capacity must be positive")
        self.capacity = int(capacity)
        self._free = [(0, self.capacity)]  # sorted, disjoint (offset, size)
        self._used = {}

    def alloc(self, nbytes: int):
        """Offset of a free range of at least nbytes, or None if none fits."""
        size = -(-int(nbytes) // self.ALIGN) * self.ALIGN
        if size <= 0:
            size = self.ALIGN
        for i, (off, avail) in enumerate(self._free):
            if avail >= size:
                if avail == size:
                    del self._free[i]
                else:
                    self._free[i] = (off + size, avail - size)
                self._used[off] = size
                return off
        return None

    def free(self, off: int) -> None:
        size = self._used.pop(off)
        self._free.append((off, size))
        self._free.sort()
        merged = []
        for o, s in self._free:
            if merged and merged[-1][0] + merged[-1][1] == o:
                merged[-1] = (merged[-1][0], merged[-1][1] + s)
            else:
                merged.append((o, s))
        self._free = merged

    @property
    def in_use(self) -> int:
        return sum(self._used.values())


class Server:
    """Continuous-batching request loop.

    executor(req, slot, offset) enqueues request ``req`` on slot ``slot`` with
    workspace at byte ``offset`` of the pool and returns a handle;
    poll(handle) returns None while it runs and (shifts, errs) once done.
    """

    def __init__(self, pool_bytes: int, slots: int, executor: Callable, poll: Callable,
                 clock: Callable[[], float] = time.perf_counter, sleep: Callable[[float], None] = time.sleep,
                 idle_sleep: float = 50e-6):
        if slots < 1:
            raise ValueError("at least one slot")
        self.pool = FootprintPool(pool_bytes)
        self.slots = slots
        self.executor = executor
        self.poll = poll
        self.clock = clock
        self.sleep = sleep
        self.idle_sleep = idle_sleep
        self.max_in_flight = 0

    def run(self, requests) -> list:
        """Serve requests (any order; each has an arrival time) in real time."""
        for r in requests:
            if r.workspace_bytes > self.pool.capacity:
                raise ValueError(f"request {r.rid} needs {r.workspace_bytes} bytes, "
                                 f"more than the pool's {self.pool.capacity}")
        pending = collections.deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
        waiting = collections.deque()
        free_slots = list(range(self.slots - 1, -1, -1))
        in_flight = []  # (req, slot, offset, handle, admitted)
        results = []
        t0 = self.clock()
        while pending or waiting or in_flight:
            now = self.clock() - t0
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            progressed = False
            still = []
            for item in in_flight:
                req, slot, off, handle, admitted = item
                out = self.poll(handle)
                if out is None:
                    still.append(item)
                    continue
                done = self.clock() - t0
                self.pool.free(off)
                free_slots.append(slot)
                results.append(Result(req.rid, req.arrival, admitted, done, out[0], out[1]))
                progressed = True
            in_flight = still
            # Admission in arrival order: a request that does not fit waits for
            # memory to free up (no overtaking, so no starvation).
            while waiting and free_slots:
                req = waiting[0]
                off = self.pool.alloc(req.workspace_bytes)
                if off is None:
                    break
                waiting.popleft()
                slot = free_slots.pop()
                admitted = self.clock() - t0
                handle = self.executor(req, slot, off)
                in_flight.append((req, slot, off, handle, admitted))
                progressed = True
            self.max_in_flight = max(self.max_in_flight, len(in_flight))
            if not progressed:
                if not in_flight and not waiting and pending:
                    wait = pending[0].arrival - (self.clock() - t0)
                    if wait > 0:
                        self.sleep(min(wait, 0.01))
                else:
                    self.sleep(self.idle_sleep)
        results.sort(key=lambda r: r.rid)
        return results


def percentile(values, q: float) -> float:
    """q-th percentile (0..100) by linear interpolation between order statistics."""
    v = sorted(values)
    if not v:
        return float("nan")
    pos = (len(v) - 1) * q / 100.0
    lo = int(pos)
    hi = min(lo + 1, len(v) - 1)
    return v[lo] + (v[hi] - v[lo]) * (pos - lo)


STAGE_ALIGN = 256


STAGE_WIDEN = 3  # pixels a staged row may gain on either side (see widen_for_dma)


def staged_image_bytes(width: int, height: int) -> int:
    """Device bytes one host-staged RGB image takes in a request's footprint
    (room for the widening of widen_for_dma)."""
    return -(-3 * (int(width) + 2 * STAGE_WIDEN) * int(height) // STAGE_ALIGN) * STAGE_ALIGN


def widen_for_dma(im):
    """(view, col): a view of the same rows as the host crop ``im`` widened to
    whole groups of four pixels of its frame, and the column of ``im`` in it.

    A host-to-device 2-D copy runs at full link speed only when its start
    addresses, row pitches and row length are multiples of 4 bytes; otherwise
    it has been measured to go row by row at a tenth of that or less.  A crop
    of a frame whose rows are a multiple of 4 bytes long starts at byte 3x of a
    row; widening it to columns [x - x % 4, ceil4(x + w)) makes every offset a
    multiple of 4.  Returns (im, 0) when the frame does not allow it.
    """
    h, w = int(im.shape[0]), int(im.shape[1])
    rs = int(im.stride(0))                 # the frame's row length in bytes
    off = int(im.storage_offset())
    frame_w = rs // 3
    x_byte = off % rs                      # where the crop starts within its row
    if rs % 12 != 0 or x_byte % 3 != 0:    # rows of whole 4-pixel groups, crop on a pixel
        return im, 0
    x = x_byte // 3
    row_start = im.data_ptr() - 3 * x      # address of the frame row's first byte
    if row_start % 4 != 0:
        return im, 0
    xa = x - x % 4
    xe = -(-(x + w) // 4) * 4
    if xe > frame_w:
        return im, 0
    view = im.as_strided((h, xe - xa, 3), (rs, 3, 1), off - 3 * (x - xa))
    return view, x - xa


def plain_workspace_bytes(mtb, n: int, width: int, height: int, levels: int) -> int:
    """Workspace of a stack run as plain per-image and per-pair calls: n pyramid
    buffers, n bitmaps buffers and n - 1 pair-search workspaces."""
    pyr = int(mtb.mtb_pyramid_bytes(width, height, levels))
    bms = int(mtb.mtb_bitmaps_bytes(width, height, levels))
    pws = int(mtb.mtb_pair_workspace_bytes(levels))
    if min(pyr, bms, pws) <= 0 or n < 1:
        raise ValueError("invalid stack request")
    return n * (pyr + bms) + (n - 1) * pws


def footprint_bytes(mtb, n: int, width: int, height: int, levels: int, host_staged: bool = False,
                    plain: bool = False) -> int:
    """Device bytes a stack request holds while in flight: its workspace (that of
    mtb_align_stack, or with plain that of the per-image and per-pair calls), and
    for a host-staged request the device copies of its n images in front of it."""
    ws = (plain_workspace_bytes(mtb, n, width, height, levels) if plain
          else int(mtb.mtb_stack_workspace_bytes(n, width, height, levels)))
    if ws <= 0:
        raise ValueError("invalid stack request")
    return ws + (n * staged_image_bytes(width, height) if host_staged else 0)


def _plain_stack(mtb, images, req, ws, shifts, errs, stream):
    """One stack as plain calls: every image's pyramid and bitmaps, then every
    moving image against the reference (the reference's row stays (0, 0), 0)."""
    n = len(images)
    h, w = int(images[0].shape[0]), int(images[0].shape[1])
    L = req.levels
    ref = req.ref_index if req.ref_index >= 0 else n // 2
    pyr = int(mtb.mtb_pyramid_bytes(w, h, L))
    bms = int(mtb.mtb_bitmaps_bytes(w, h, L))
    pws = int(mtb.mtb_pair_workspace_bytes(L))
    shifts.zero_()
    errs.zero_()
    bitmaps = []
    for i, im in enumerate(images):
        p = ws[i * pyr:(i + 1) * pyr]
        b = ws[n * pyr + i * bms:n * pyr + (i + 1) * bms]
        mtb.mtb_build_pyramid(im, L, pyramid=p, stream=stream)
        mtb.mtb_bitmaps(p, w, h, L, exclude_range=req.exclude_range, bitmaps=b, stream=stream)
        bitmaps.append(b)
    base = n * (pyr + bms)
    k = 0
    for i in range(n):
        if i == ref:
            continue
        mtb.mtb_align_pair(bitmaps[ref], bitmaps[i], w, h, L, workspace=ws[base + k * pws:base + (k + 1) * pws],
                           shift=shifts[i], err=errs[i:i + 1], stream=stream)
        k += 1


def gpu_executor(pool_buffer, slots: int, plain: bool = False):
    """Executor and poll functions that run requests through libmtb on `slots` streams.

    pool_buffer is a uint8 device tensor holding the serving pool; request
    footprints are views into it.  A request whose images are CPU tensors is
    host-staged: its footprint starts with one device image per input (see
    footprint_bytes), filled by mtb_stage_rgb on the slot's stream, and the
    workspace follows.  Streams are created at default priority.  With plain
    (the per-call path, for comparison) a stack runs as mtb_build_pyramid and
    mtb_bitmaps per image and mtb_align_pair per moving image, each its own
    launch sequence, instead of one mtb_align_stack call; the results are the
    same.
    """
    import torch

    import paper_2007_06483_amd as mtb

    streams = [torch.cuda.Stream(device=pool_buffer.device) for _ in range(slots)]

    def execute(req, slot, off):
        s = streams[slot]
        # Inputs were produced on the current stream; the slot's stream waits for them.
        s.wait_stream(torch.cuda.current_stream(pool_buffer.device))
        images = req.images
        ws_off = off
        if images[0].device.type == "cpu":
            # The images of a stack share one row stride: every staged copy gets
            # rows as long as the widest widened crop.
            widened = [widen_for_dma(im) for im in req.images]
            wmax = max(int(v.shape[1]) for v, _ in widened)
            images = []
            for im, (src, col) in zip(req.images, widened):
                h, w = int(im.shape[0]), int(im.shape[1])
                dst = pool_buffer[ws_off:ws_off + 3 * wmax * h].view(h, wmax, 3)
                mtb.mtb_stage_rgb(src, dst[:, :int(src.shape[1])], stream=s)
                images.append(dst[:, col:col + w])
                ws_off += staged_image_bytes(w, h)
        ws = pool_buffer[ws_off:off + req.workspace_bytes]
        n = len(images)
        with torch.cuda.stream(s):
            shifts = torch.empty((n, 2), dtype=torch.int32, device=pool_buffer.device)
            errs = torch.empty(n, dtype=torch.int32, device=pool_buffer.device)
            if plain:
                _plain_stack(mtb, images, req, ws, shifts, errs, s)
            else:
                mtb.mtb_align_stack(images, req.levels, exclude_range=req.exclude_range,
                                    ref_index=req.ref_index, workspace=ws, shifts=shifts, errs=errs,
                                    stream=s)
            ev = torch.cuda.Event()
            ev.record(s)
        return (ev, shifts, errs)

    def poll(handle):
        ev, shifts, errs = handle
        if not ev.query():
            return None
        return shifts, errs

    return execute, poll
