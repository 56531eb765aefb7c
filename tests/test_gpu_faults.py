"""Failed launches (injected from the host, so no kernel ever faults): the call
that hits one returns MTB_ERR_DEVICE, and the next call on the same workspace
and outputs is bit-exact again, wherever in the launch sequence the failure
fell."""

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
    yield m
    m.mtb_test_fail_launch(-1)


def _launch_count(mtb, fn):
    mtb.mtb_profile_begin(None)
    fn()
    torch.cuda.synchronize()
    return sum(c for c, _ in mtb.mtb_profile_end().values())


def test_stack_recovers_after_a_failed_launch_anywhere(mtb):
    imgs, _, _ = synth.make_stack(700, 500, 4, 30, 71, 20)
    L = 5
    d = [torch.from_numpy(im).to(DEV) for im in imgs]
    want = oracle.align_stack(imgs, L, threads=4)
    ws = torch.empty(mtb.mtb_stack_workspace_bytes(4, 700, 500, L), dtype=torch.uint8, device=DEV)
    sh = torch.empty((4, 2), dtype=torch.int32, device=DEV)
    er = torch.empty(4, dtype=torch.int32, device=DEV)

    def call():
        return mtb.mtb_align_stack(d, L, workspace=ws, shifts=sh, errs=er)

    n = _launch_count(mtb, call)
    assert n >= 5
    for after in range(n):
        mtb.mtb_test_fail_launch(after)
        with pytest.raises(RuntimeError, match="MTB_ERR_DEVICE"):
            call()
        torch.cuda.synchronize()
        call()
        torch.cuda.synchronize()
        assert np.array_equal(sh.cpu().numpy(), want["shifts"]), after
        assert np.array_equal(er.cpu().numpy().astype(np.int64), want["errs"]), after
    # A failure scheduled past the end of one call lands in the next one.
    mtb.mtb_test_fail_launch(n)
    call()
    with pytest.raises(RuntimeError, match="MTB_ERR_DEVICE"):
        call()
    mtb.mtb_test_fail_launch(-1)
    call()
    torch.cuda.synchronize()
    assert np.array_equal(sh.cpu().numpy(), want["shifts"])


def test_batch_recovers_after_a_failed_launch_in_a_later_group(mtb):
    items = []
    for k, (w, h, L) in enumerate([(200, 150, 4), (321, 243, 5), (200, 150, 4)]):
        ref, mov, _ = synth.make_rect_pair(w, h, 12, 880 + k, (1 << (L - 1)) - 1)
        items.append((ref, mov, L))
    dev = [(torch.from_numpy(r).to(DEV), torch.from_numpy(m).to(DEV), L) for r, m, L in items]
    want = np.array([oracle.align_pair(r, m, L)["shift"] for r, m, L in items], dtype=np.int32)
    n = _launch_count(mtb, lambda: mtb.mtb_align_batch(dev))
    for after in (n // 2, n - 1):
        mtb.mtb_test_fail_launch(after)
        with pytest.raises(RuntimeError, match="MTB_ERR_DEVICE"):
            mtb.mtb_align_batch(dev)
        torch.cuda.synchronize()
        got = mtb.mtb_align_batch(dev)
        torch.cuda.synchronize()
        assert np.array_equal(got["shifts"].cpu().numpy(), want), after


def test_tuner_failure_stores_no_shape(mtb):
    imgs, _, _ = synth.make_stack(400, 300, 3, 20, 72, 10)
    d = [torch.from_numpy(im).to(DEV) for im in imgs]
    mtb.mtb_tune_reset()
    mtb.mtb_test_fail_launch(30)   # inside the tuner's timed trials
    with pytest.raises(RuntimeError, match="MTB_ERR_DEVICE"):
        mtb.mtb_tune_stack(d, 4)
    torch.cuda.synchronize()
    assert mtb.mtb_tuned_shape(3, 400, 300, 1200, 4) is None
    mtb.mtb_test_fail_launch(-1)
    shape = mtb.mtb_tune_stack(d, 4)
    assert mtb.mtb_tuned_shape(3, 400, 300, 1200, 4)["pyramid_slots_pct"] == shape["pyramid_slots_pct"]
    mtb.mtb_tune_reset()
