"""Host logic of bench.py: the one-GPU guard, the algorithmic byte model and the
rule that stored counter figures apply only to the workload and kernel sources
they were taken on."""

import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_algorithmic_bytes_of_the_stack_workload():
    import paper_2007_06483_amd as mtb

    W, H, L, n = 6000, 4000, 7, 7
    lay = mtb.mtb_get_layout(W, H, L)
    per = bench.algorithmic_bytes(lay, n, n - 1)
    gray = sum((W >> l) * (H >> l) for l in range(L))
    l1 = (W >> 1) * (H >> 1)  # level 1's gray: neither written nor read by the stack path
    maps = sum(8 * (((W >> l) + 63) // 64) * (H >> l) for l in range(L))
    assert per["k_pyramid"] == n * (3 * W * H + gray - l1) == 685985237
    assert per["k_bitmaps"] == n * (gray - l1 + 2 * maps)
    assert per["search"] == (n - 1) * 4 * maps
    assert per["step"] == per["k_pyramid"] + per["k_bitmaps"] + per["search"]
    # The staged method's yardstick: every gray level written once and read once.
    assert per["step_model"] == per["step"] + 2 * n * l1 == 1104578170
    assert bench.pyramid_bytes(W, H, L, level1=False) * n == per["k_pyramid"]
    assert bench.pyramid_bytes(W, H, L) * n == per["k_pyramid"] + n * l1


def test_stored_traffic_applies_only_to_its_own_workload(tmp_path, monkeypatch):
    f = tmp_path / "traffic.json"
    kernels = {"k_pyramid": {"traffic_bytes_per_launch": 123}, "k_bitmaps": {"traffic_bytes_per_launch": 45}}
    f.write_text(json.dumps({"workload": "stack7_6000x4000", "kernel_source_sha256": bench.kernel_source_sha256(),
                             "kernels": kernels}))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.load_traffic("stack7_6000x4000") == {"k_pyramid": 123, "k_bitmaps": 45}
    assert bench.load_traffic("stack7_6000x4000_chained") == {}    # another launch sequence
    assert bench.load_traffic("pair_4096x3072") == {}
    f.write_text(json.dumps({"workload": "stack7_6000x4000", "kernel_source_sha256": "0" * 64,
                             "kernels": kernels}))
    assert bench.load_traffic("stack7_6000x4000") == {}            # kernels changed since
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.json"))
    assert bench.load_traffic("stack7_6000x4000") == {}
