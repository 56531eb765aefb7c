"""The oracle and the generator reproduce the stored expected values in tests/golden/.

The stored values were written by tests/golden/make_golden.py, which calls
only the oracle and the generator; a mismatch means one of them changed.
"""

import json
import os

import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_pairs.json")


def _inputs(name):
    if name == "pair_512x384":
        (imgs, _, _), = synth.workload(name).stacks
        return imgs[0], imgs[1]
    if name == "rect_pair_640x480_seed5150":
        ref, mov, _ = synth.make_rect_pair(640, 480, 80, 5150, 30)
        return ref, mov
    raise KeyError(name)


@pytest.mark.parametrize("case", json.load(open(GOLDEN))["cases"], ids=lambda c: c["name"])
def test_oracle_matches_golden(case):
    ref, mov = _inputs(case["name"])
    assert synth.sha256(ref) == case["sha256_ref"]
    assert synth.sha256(mov) == case["sha256_mov"]
    r = oracle.align_pair(ref, mov, case["levels"])
    assert list(r["shift"]) == case["shift"]
    assert r["err"] == case["err"]
    assert r["trace"].tolist() == case["trace"]
    assert r["level_shifts"].tolist() == case["level_shifts"]
    assert r["ref"].median.tolist() == case["median_ref"]
    assert r["mov"].median.tolist() == case["median_mov"]
