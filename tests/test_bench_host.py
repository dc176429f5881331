"""Host logic of bench.py: the algorithmic byte count and the traffic lookup."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_algorithmic_bytes_count():
    info = {"n_nodes": 10, "n_bulk": 3, "n_pairs": 2}
    # 96 B/node + 32 B/GP + 8 B/pair in mixed precision; 64 and 16 in FP64
    assert bench.algorithmic_bytes(info, 1) == 960 + 96 + 16
    assert bench.algorithmic_bytes(info, 0) == 960 + 192 + 32


def test_traffic_needs_matching_source_and_workload(tmp_path, monkeypatch):
    f = tmp_path / "t.txt"
    f.write_text(f"workload_key: w1\nkernel_source_sha256: {bench.kernel_source_hash()}\n"
                 "traffic_bytes_per_launch: 1.5e9\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_traffic("w1") == pytest.approx(1.5e9)
    assert bench.measured_traffic("w2") is None
    f.write_text("workload_key: w1\nkernel_source_sha256: 00\ntraffic_bytes_per_launch: 1.5e9\n")
    assert bench.measured_traffic("w1") is None


def test_multi_gpu_request_exits(monkeypatch, capsys):
    monkeypatch.setattr(sys, "argv", ["bench.py", "--gpus", "2"])
    with pytest.raises(SystemExit) as e:
        bench.main()
    assert e.value.code == 2
    assert "one GPU" in capsys.readouterr().out


def test_kernel_hash_covers_every_source_of_the_element_kernel():
    """The traffic summary is tied to the element/node kernel's sources: the
    hash must cover every local file pdn_kernels.hip includes, transitively."""
    import re
    csrc = os.path.join(ROOT, "paper_2301_05552_amd", "csrc")
    seen, todo = set(), ["pdn_kernels.hip"]
    while todo:
        f = todo.pop()
        if f in seen:
            continue
        seen.add(f)
        with open(os.path.join(csrc, f)) as fh:
            for m in re.finditer(r'^\s*#include\s+"([^"]+)"', fh.read(), re.M):
                if os.path.exists(os.path.join(csrc, m.group(1))):
                    todo.append(m.group(1))
    hashed = {os.path.basename(p) for p in bench.KERNEL_SOURCES}
    assert seen <= hashed, sorted(seen - hashed)
