"""Writes the stored expected values under tests/golden/ from the CPU oracle alone.

    python tests/golden/make_golden.py

Inputs come from the seeded generator (synth); every number stored here is
produced by the oracle package and nothing else.  The tests re-derive them to
catch any unintended change to the oracle's arithmetic.
"""

import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402


def record(name, ref, mov, t, levels):
    r = oracle.align_pair(ref, mov, levels)
    return {
        "name": name,
        "width": int(ref.shape[1]),
        "height": int(ref.shape[0]),
        "levels": levels,
        "planted_translation": list(t),
        "sha256_ref": synth.sha256(ref),
        "sha256_mov": synth.sha256(mov),
        "median_ref": r["ref"].median.tolist(),
        "median_mov": r["mov"].median.tolist(),
        "shift": list(r["shift"]),
        "err": r["err"],
        "level_shifts": r["level_shifts"].tolist(),
        "trace": r["trace"].tolist(),
    }


def main():
    cases = []
    w = synth.workload("pair_512x384")
    (imgs, shifts, _), = w.stacks
    cases.append(record("pair_512x384", imgs[0], imgs[1], shifts[1], w.levels))
    ref, mov, t = synth.make_rect_pair(640, 480, 80, 5150, 30)
    cases.append(record("rect_pair_640x480_seed5150", ref, mov, t, 5))
    with open(os.path.join(HERE, "oracle_pairs.json"), "w") as f:
        json.dump({"generated_by": "tests/golden/make_golden.py (oracle only)", "cases": cases}, f,
                  indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
