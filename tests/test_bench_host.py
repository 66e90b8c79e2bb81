"""Host logic of bench.py (no GPU): the one-GPU guard, the algorithmic
byte/flop model behind the roofline, and the lookup of stored traffic
readings, which must be dropped once the stage kernel's sources change."""
import json
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "error" in line and line["n_gpus"] == 2


def test_stage_model_counts():
    h, w, N, R = 64, 32, 6, 15
    px = h * w
    m = bench.stage_model(h, w, "gaussian", R, N, 4, True)
    # the stack kernel reads f once and writes alpha, beta and N FP32 planes
    assert m["stack"]["bytes"] == px * (4 + 8 + 4 * N)
    # two separable passes of 2R+1 FMAs per power, 2 flops each
    conv = 4 * N * (2 * R + 1)
    shift = N * (N + 1) + 2 * N + (N * N) // 2
    assert m["stack"]["flops"] == px * (conv + shift)
    assert m["moments"] == m["stack"]
    assert m["minmax"]["bytes"] == px * 12 and m["minmax"]["flops"] == 0
    # the range stage reads alpha, beta, N moments, theta and sigma, writes out
    assert m["range"]["bytes"] == px * (8 + 4 * N + 4 + 4 + 4)
    box = bench.stage_model(h, w, "box", 5, N, 4, False)
    assert box["moments"]["flops"] == px * (4 * N + shift)


def test_traffic_lookup_follows_the_sources(tmp_path, monkeypatch):
    root = tmp_path / "repo"
    csrc = root / "paper_1811_02308_amd" / "csrc"
    csrc.mkdir(parents=True)
    for name in {n for srcs in bench.STAGE_SOURCES.values() for n in srcs}:
        shutil.copy(os.path.join(ROOT, "paper_1811_02308_amd", "csrc", name), csrc / name)
    (root / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(root))
    h = bench.stage_source_hash("stack")
    assert h == bench.stage_source_hash("moments")          # same kernel sources
    assert h == bench.stage_source_hash("moments_range")
    assert h != bench.stage_source_hash("range")
    table = ("| workload | stage | kernel | FETCH_SIZE KiB | WRITE_SIZE KiB | FETCH scale | "
             "WRITE scale | bytes | source |\n|---|---|---|---|---|---|---|---|---|\n"
             f"| wl | stack | `k` | 1 | 2 | 2.000 | 1.000 | 12345 | {h} |\n")
    (root / "profiles" / "traffic.md").write_text(table)
    assert bench.measured_traffic("wl", "stack") == 12345
    assert bench.measured_traffic("wl", "range") is None
    assert bench.measured_traffic("other", "stack") is None
    # any change to the kernel's sources invalidates the reading, the shared
    # device helpers included
    with open(csrc / "moments_common.h", "a") as fh:
        fh.write("\n// changed\n")
    assert bench.measured_traffic("wl", "stack") is None
