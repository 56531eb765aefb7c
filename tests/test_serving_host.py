"""Host logic of the serving loop: footprint pool and continuous-batching admission.

Runs on the CPU with a simulated clock and an executor whose requests finish
after a fixed time, so admission, overlap and retirement are checked exactly.
"""

import pytest

from paper_2007_06483_amd.serving import FootprintPool, Request, Server, percentile


def test_pool_first_fit_alignment_and_merge():
    p = FootprintPool(4096)
    a = p.alloc(100)
    b = p.alloc(256)
    c = p.alloc(1)
    assert (a, b, c) == (0, 256, 512)
    assert p.in_use == 768
    assert p.alloc(4096) is None
    p.free(b)
    assert p.alloc(200) == 256          # first fit reuses the hole
    p.free(a)
    p.free(256)
    p.free(c)
    assert p.in_use == 0
    assert p.alloc(4096) == 0           # holes merged back into one range


def test_pool_rejects_bad_capacity():
    with pytest.raises(ValueError):
        FootprintPool(0)


class Sim:
    """Simulated time: sleep advances it; requests finish `dur` after admission."""

    def __init__(self, dur):
        self.now = 0.0
        self.dur = dur
        self.active = 0
        self.peak = 0

    def clock(self):
        return self.now

    def sleep(self, dt):
        self.now += max(dt, 1e-6)

    def execute(self, req, slot, off):
        self.active += 1
        self.peak = max(self.peak, self.active)
        return {"req": req, "end": self.now + self.dur[req.rid], "slot": slot, "off": off, "done": False}

    def poll(self, h):
        if self.now < h["end"]:
            return None
        if not h["done"]:
            h["done"] = True
            self.active -= 1
        return ("shifts", h["req"].rid), ("errs", h["req"].rid)


def _req(rid, arrival, ws):
    return Request(rid=rid, arrival=arrival, images=[], levels=1, workspace_bytes=ws)


def test_requests_arriving_during_work_are_admitted_at_once():
    # Two slots, plenty of memory: request 1 arrives while 0 runs and starts
    # immediately (continuous batching), not after 0 completes.
    sim = Sim({0: 1.0, 1: 1.0, 2: 0.5})
    srv = Server(1 << 20, 2, sim.execute, sim.poll, clock=sim.clock, sleep=sim.sleep, idle_sleep=1e-3)
    res = srv.run([_req(0, 0.0, 1000), _req(1, 0.3, 1000), _req(2, 0.4, 1000)])
    r0, r1, r2 = res
    assert r1.admitted == pytest.approx(0.3, abs=2e-3)
    assert r1.admitted < r0.completed
    # The third waits for a free slot: it starts when request 0 finishes.
    assert r2.admitted == pytest.approx(r0.completed, abs=2e-3)
    assert sim.peak == 2 and srv.max_in_flight == 2
    for r, d in zip(res, (1.0, 1.0, 0.5)):
        assert r.completed - r.admitted == pytest.approx(d, abs=2e-3)
        assert r.shifts == ("shifts", r.rid)


def test_admission_by_footprint_waits_for_memory_in_arrival_order():
    # Pool of 3000 bytes, four slots: the 2000-byte request must wait for the
    # first to free memory; the small one behind it does not overtake it.
    sim = Sim({0: 1.0, 1: 1.0, 2: 0.1})
    srv = Server(3000, 4, sim.execute, sim.poll, clock=sim.clock, sleep=sim.sleep, idle_sleep=1e-3)
    res = srv.run([_req(0, 0.0, 2000), _req(1, 0.1, 2000), _req(2, 0.2, 256)])
    assert res[1].admitted == pytest.approx(res[0].completed, abs=2e-3)
    assert res[2].admitted >= res[1].admitted
    assert srv.pool.in_use == 0


def test_oversized_request_is_refused():
    sim = Sim({0: 1.0})
    srv = Server(1000, 1, sim.execute, sim.poll, clock=sim.clock, sleep=sim.sleep)
    with pytest.raises(ValueError):
        srv.run([_req(0, 0.0, 5000)])


def test_percentile_interpolates():
    assert percentile([1, 2, 3, 4], 50) == pytest.approx(2.5)
    assert percentile([5], 99) == 5
    assert percentile(list(range(101)), 99) == pytest.approx(99)


def test_host_staged_footprint_holds_the_images_before_the_workspace():
    import paper_2007_06483_amd as mtb
    from paper_2007_06483_amd.serving import footprint_bytes, staged_image_bytes

    assert staged_image_bytes(1, 1) == 256           # 7 pixels with the widening
    assert staged_image_bytes(58, 4) == 768          # 3 * 64 * 4 bytes, already aligned
    assert staged_image_bytes(59, 4) == 1024         # 780 bytes rounded up
    n, w, h, L = 5, 1000, 700, 6
    ws = mtb.mtb_stack_workspace_bytes(n, w, h, L)
    assert footprint_bytes(mtb, n, w, h, L) == ws
    assert footprint_bytes(mtb, n, w, h, L, host_staged=True) == ws + n * staged_image_bytes(w, h)
    with pytest.raises(ValueError):
        footprint_bytes(mtb, 0, w, h, L)
    # The per-call comparison path: n pyramids, n bitmaps, n - 1 pair workspaces.
    plain = footprint_bytes(mtb, n, w, h, L, plain=True)
    assert plain == n * (mtb.mtb_pyramid_bytes(w, h, L) + mtb.mtb_bitmaps_bytes(w, h, L)) + \
        (n - 1) * mtb.mtb_pair_workspace_bytes(L)
    assert footprint_bytes(mtb, n, w, h, L, host_staged=True, plain=True) == plain + n * staged_image_bytes(w, h)


def test_widen_for_dma_aligns_every_offset_and_keeps_the_crop():
    import numpy as np
    import torch

    from paper_2007_06483_amd.serving import STAGE_WIDEN, widen_for_dma

    frame = torch.from_numpy(np.random.default_rng(3).integers(0, 256, (40, 100, 3), dtype=np.uint8))
    for x in range(0, 12):
        for w in (1, 5, 17, 60, 100 - x):
            crop = frame[7:30, x:x + w]
            view, col = widen_for_dma(crop)
            assert torch.equal(view[:, col:col + w], crop), (x, w)
            ww = view.shape[1]
            assert ww <= w + 2 * STAGE_WIDEN
            assert view.stride(0) == 300 and (view.data_ptr() - frame.data_ptr()) % 4 == 0
            assert (3 * ww) % 4 == 0 and view.data_ptr() % 4 == 0
    # A frame whose rows are not a multiple of 4 bytes long is left alone.
    odd = torch.zeros((10, 33, 3), dtype=torch.uint8)
    v, col = widen_for_dma(odd[2:5, 3:9])
    assert col == 0 and v.shape[1] == 6
