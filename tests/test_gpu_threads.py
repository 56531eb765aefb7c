"""Several host threads calling the library at once, each on its own stream
with its own workspace: every result equals the same stack aligned alone."""

import threading

import numpy as np
import pytest

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


def test_threads_on_their_own_streams_match_results_alone(mtb):
    stacks = []
    for k, (w, h, n, L) in enumerate([(640, 480, 3, 5), (1000, 700, 5, 6), (321, 243, 4, 4), (1500, 900, 3, 6)]):
        imgs, _, _ = synth.make_stack(w, h, n, 30, 500 + k, 12, sat_frac=0.02)
        stacks.append(([torch.from_numpy(im).to(DEV) for im in imgs], L))
    alone = []
    for d, L in stacks:
        r = mtb.mtb_align_stack(d, L, trace=True)
        torch.cuda.synchronize()
        alone.append((r["shifts"].cpu().numpy(), r["errs"].cpu().numpy(), r["trace"].cpu().numpy()))

    got = [[] for _ in stacks]
    errors = []

    def work(i):
        try:
            d, L = stacks[i]
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                for _ in range(3):
                    r = mtb.mtb_align_stack(d, L, trace=True, stream=s)
                    s.synchronize()
                    got[i].append((r["shifts"].cpu().numpy(), r["errs"].cpu().numpy(),
                                   r["trace"].cpu().numpy()))
        except Exception as e:  # reported below, on the main thread
            errors.append((i, repr(e)))

    threads = [threading.Thread(target=work, args=(i,)) for i in range(len(stacks))]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=120)
    assert not any(t.is_alive() for t in threads)
    assert not errors, errors
    for i, runs in enumerate(got):
        assert len(runs) == 3
        for run in runs:
            for a, b in zip(alone[i], run):
                assert np.array_equal(a, b), i
