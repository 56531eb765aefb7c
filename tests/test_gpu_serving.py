"""Served alignment on the GPU: each stack's result in the mix equals its result alone.

Requests are cut from a small base scene and arrive as a Poisson stream with
an initial burst, so several stacks are in flight at once on different
streams with workspaces from one pool.  Every served result must equal the
result of aligning that stack alone (bit-exact), and a sample must equal the
oracle.
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


@pytest.mark.timeout(600)
def test_served_results_equal_results_alone(mtb):
    from paper_2007_06483_amd.serving import Request, Server, gpu_executor

    BW, BH = 1536, 1024
    base = synth.make_serve_base(BW, BH, 6, n_blobs=60)
    base_dev = [torch.from_numpy(b).to(DEV) for b in base]
    specs = synth.serve_requests(7, 400.0, 0.15, BW, BH, mp_range=(0.05, 0.6))
    assert len(specs) >= 20
    reqs = []
    for k, r in enumerate(specs):
        imgs = [synth.serve_crop(base_dev, r, i) for i in range(r["n"])]
        ws = mtb.mtb_stack_workspace_bytes(r["n"], r["width"], r["height"], r["levels"])
        # The first eight arrive together: a burst that fills every slot.
        reqs.append(Request(rid=r["rid"], arrival=0.0 if k < 8 else r["arrival"], images=imgs,
                            levels=r["levels"], workspace_bytes=ws))
    slots = 4
    pool_bytes = slots * max(q.workspace_bytes for q in reqs) + 4096
    pool = torch.empty(pool_bytes, dtype=torch.uint8, device=DEV)
    execute, poll = gpu_executor(pool, slots)
    srv = Server(pool_bytes, slots, execute, poll)
    results = srv.run(reqs)
    torch.cuda.synchronize()
    assert len(results) == len(reqs)
    assert srv.max_in_flight > 1
    for q, res in zip(reqs, results):
        alone = mtb.mtb_align_stack(q.images, q.levels)
        torch.cuda.synchronize()
        assert torch.equal(res.shifts, alone["shifts"]), q.rid
        assert torch.equal(res.errs, alone["errs"]), q.rid
        assert res.completed >= res.admitted >= res.arrival - 1e-9
    for r in specs[:: max(1, len(specs) // 5)]:
        host = [np.ascontiguousarray(synth.serve_crop(base, r, i)) for i in range(r["n"])]
        want = oracle.align_stack(host, r["levels"], ref_index=r["n"] // 2, threads=4)
        got = results[r["rid"]]
        assert np.array_equal(got.shifts.cpu().numpy(), want["shifts"]), r["rid"]
        assert np.array_equal(got.errs.cpu().numpy().astype(np.int64), want["errs"]), r["rid"]


@pytest.mark.timeout(900)
def test_served_full_size_requests(mtb):
    """Requests at the served workload's own ranges: 3-9 exposures of 1-48 MP
    (log-uniform, 3:2), up to 7 levels, cut from the 8704x5888 nine-exposure base
    scene.  The first eight arrive together, five of them 8 MP or more, so several
    large stacks are in flight at once.  Every result must equal that stack
    aligned alone, and a seeded sample of eight (the four largest and four drawn
    from the rest) must equal the oracle's."""
    import concurrent.futures

    from paper_2007_06483_amd.serving import Request, Server, gpu_executor

    BW, BH = 8704, 5888
    base = synth.make_serve_base(BW, BH, 5)
    base_dev = [torch.from_numpy(b).to(DEV) for b in base]
    specs = synth.serve_requests(26, 200.0, 0.15, BW, BH)
    assert len(specs) >= 30
    assert max(r["width"] * r["height"] for r in specs) > 40e6
    reqs = []
    for k, r in enumerate(specs):
        imgs = [synth.serve_crop(base_dev, r, i) for i in range(r["n"])]
        ws = mtb.mtb_stack_workspace_bytes(r["n"], r["width"], r["height"], r["levels"])
        reqs.append(Request(rid=r["rid"], arrival=0.0 if k < 8 else r["arrival"], images=imgs,
                            levels=r["levels"], workspace_bytes=ws))
    slots = 8
    pool_bytes = slots * max(q.workspace_bytes for q in reqs) + 4096
    pool = torch.empty(pool_bytes, dtype=torch.uint8, device=DEV)
    execute, poll = gpu_executor(pool, slots)
    srv = Server(pool_bytes, slots, execute, poll)
    results = srv.run(reqs)
    torch.cuda.synchronize()
    assert len(results) == len(reqs)
    # At least three stacks of 8 MP or more overlapped in time.
    big = [res for res, r in zip(results, specs) if r["width"] * r["height"] >= 8e6]
    overlap = max(sum(1 for o in big if o.admitted <= b.admitted < o.completed) for b in big)
    assert overlap >= 3, overlap
    for q, res in zip(reqs, results):
        alone = mtb.mtb_align_stack(q.images, q.levels)
        torch.cuda.synchronize()
        assert torch.equal(res.shifts, alone["shifts"]), q.rid
        assert torch.equal(res.errs, alone["errs"]), q.rid
    del pool, base_dev
    order = sorted(range(len(specs)), key=lambda k: -specs[k]["width"] * specs[k]["height"] * specs[k]["n"])
    rest = np.random.default_rng(26).choice(order[4:], 4, replace=False)
    sample = order[:4] + sorted(int(k) for k in rest)

    def one(k):
        r = specs[k]
        host = [np.ascontiguousarray(synth.serve_crop(base, r, i)) for i in range(r["n"])]
        return oracle.align_stack(host, r["levels"], ref_index=r["n"] // 2, threads=2)

    with concurrent.futures.ThreadPoolExecutor(max_workers=4) as ex:
        wants = list(ex.map(one, sample))
    for k, want in zip(sample, wants):
        got = results[specs[k]["rid"]]
        assert np.array_equal(got.shifts.cpu().numpy(), want["shifts"]), k
        assert np.array_equal(got.errs.cpu().numpy().astype(np.int64), want["errs"]), k


def test_stage_rgb_copies_a_strided_host_view(mtb):
    base = torch.from_numpy(np.random.default_rng(11).integers(0, 256, (70, 150, 3), dtype=np.uint8)).pin_memory()
    view = base[5:65, 7:140]                       # rows 450 bytes apart, 133 pixels used
    dst_buf = torch.full((60, 141, 3), 7, dtype=torch.uint8, device=DEV)
    dst = dst_buf[:, :133]                         # device rows 423 bytes apart
    mtb.mtb_stage_rgb(view, dst)
    torch.cuda.synchronize()
    assert torch.equal(dst.cpu(), view)
    assert bool((dst_buf[:, 133:] == 7).all())     # bytes past the row untouched


@pytest.mark.timeout(600)
def test_host_staged_serving_equals_device_staged(mtb):
    from paper_2007_06483_amd.serving import Request, Server, footprint_bytes, gpu_executor

    BW, BH = 1200, 800
    base = synth.make_serve_base(BW, BH, 8, n_blobs=50)
    base_host = [torch.from_numpy(b).pin_memory() for b in base]
    base_dev = [torch.from_numpy(b).to(DEV) for b in base]
    specs = synth.serve_requests(9, 300.0, 0.1, BW, BH, mp_range=(0.05, 0.4))
    assert len(specs) >= 10

    def requests(src, host):
        return [Request(rid=r["rid"], arrival=0.0 if k < 6 else r["arrival"],
                        images=[synth.serve_crop(src, r, i) for i in range(r["n"])], levels=r["levels"],
                        workspace_bytes=footprint_bytes(mtb, r["n"], r["width"], r["height"], r["levels"], host))
                for k, r in enumerate(specs)]

    out = {}
    for host in (False, True):
        reqs = requests(base_host if host else base_dev, host)
        slots = 3
        pool_bytes = slots * max(q.workspace_bytes for q in reqs) + 4096
        pool = torch.empty(pool_bytes, dtype=torch.uint8, device=DEV)
        execute, poll = gpu_executor(pool, slots)
        srv = Server(pool_bytes, slots, execute, poll)
        out[host] = srv.run(reqs)
        torch.cuda.synchronize()
        assert srv.max_in_flight > 1
    for a, b in zip(out[False], out[True]):
        assert a.rid == b.rid
        assert torch.equal(a.shifts, b.shifts), a.rid
        assert torch.equal(a.errs, b.errs), a.rid
    r = specs[len(specs) // 2]
    host = [np.ascontiguousarray(synth.serve_crop(base, r, i)) for i in range(r["n"])]
    want = oracle.align_stack(host, r["levels"], ref_index=r["n"] // 2, threads=4)
    assert np.array_equal(out[True][r["rid"]].shifts.cpu().numpy(), want["shifts"])


@pytest.mark.timeout(600)
def test_plain_per_call_serving_equals_stack_serving(mtb):
    """The per-call comparison path of the served bench (per-image pyramid and
    bitmaps calls, one pair call per moving image) serves the same requests
    with the same results as one mtb_align_stack call per request."""
    from paper_2007_06483_amd.serving import Request, Server, footprint_bytes, gpu_executor

    BW, BH = 1400, 900
    base = synth.make_serve_base(BW, BH, 12, n_blobs=60)
    base_dev = [torch.from_numpy(b).to(DEV) for b in base]
    specs = synth.serve_requests(13, 300.0, 0.1, BW, BH, mp_range=(0.05, 0.6))
    assert len(specs) >= 10
    out = {}
    for plain in (False, True):
        reqs = [Request(rid=r["rid"], arrival=0.0 if k < 6 else r["arrival"],
                        images=[synth.serve_crop(base_dev, r, i) for i in range(r["n"])], levels=r["levels"],
                        workspace_bytes=footprint_bytes(mtb, r["n"], r["width"], r["height"], r["levels"],
                                                        plain=plain))
                for k, r in enumerate(specs)]
        slots = 4
        pool_bytes = slots * max(q.workspace_bytes for q in reqs) + 4096
        pool = torch.empty(pool_bytes, dtype=torch.uint8, device=DEV)
        execute, poll = gpu_executor(pool, slots, plain=plain)
        srv = Server(pool_bytes, slots, execute, poll)
        out[plain] = srv.run(reqs)
        torch.cuda.synchronize()
        assert srv.max_in_flight > 1
    for a, b in zip(out[False], out[True]):
        assert a.rid == b.rid
        assert torch.equal(a.shifts, b.shifts), a.rid
        assert torch.equal(a.errs, b.errs), a.rid
    r = specs[len(specs) // 3]
    host = [np.ascontiguousarray(synth.serve_crop(base, r, i)) for i in range(r["n"])]
    want = oracle.align_stack(host, r["levels"], ref_index=r["n"] // 2, threads=4)
    assert np.array_equal(out[True][r["rid"]].shifts.cpu().numpy(), want["shifts"])
    assert np.array_equal(out[True][r["rid"]].errs.cpu().numpy().astype(np.int64), want["errs"])
