"""Host-side checks of the measurement plumbing in bench.py: the algorithmic
byte model, and the committed HBM-traffic summary that the bench line quotes
(its arithmetic, and that it is only reported for the kernel source it was
measured on)."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _traffic_fields():
    kv = {}
    with open(bench.TRAFFIC_FILE) as f:
        for line in f:
            line = line.strip()
            if "=" in line and not line.startswith("#"):
                k, v = line.split("=", 1)
                kv[k.strip()] = v.strip()
    return kv


def test_algorithmic_bytes_per_cell():
    # read the interior and the 2d face-halo layers, write the interior:
    # ((p^d + 2d p^(d-1)) s + p^d s) e / p^d
    assert bench.algorithmic_bytes_per_cell(3, 8, 5, 8) == 110.0
    assert bench.algorithmic_bytes_per_cell(3, 8, 5, 4) == 55.0
    assert bench.algorithmic_bytes_per_cell(2, 16, 4, 8) == 72.0
    assert bench.algorithmic_bytes_per_cell(3, 16, 5, 8) == 95.0
    assert bench.algorithmic_bytes_per_cell(3, 4, 5, 8) == 140.0


def test_traffic_summary_is_consistent():
    kv = _traffic_fields()
    fetch = float(kv["fetch_size_kib_per_dispatch"]) * 1024 * float(kv["fetch_scale"])
    write = float(kv["write_size_kib_per_dispatch"]) * 1024 * float(kv["write_scale"])
    assert abs(fetch - float(kv["l2_fabric_read_bytes_per_launch"])) <= 1e-3 * fetch
    assert abs(write - float(kv["l2_fabric_write_bytes_per_launch"])) <= 1e-3 * write
    total = float(kv["l2_fabric_bytes_per_launch"])
    assert abs(total - fetch - write) <= 1e-3 * total
    alg = float(kv["algorithmic_bytes_per_launch"])
    assert alg == bench.algorithmic_bytes_per_cell(3, 8, 5, 8) * 4096 * 8 ** 3
    assert abs(float(kv["traffic_over_algorithmic"]) - total / alg) <= 1e-3
    # the write counter of a plain copy reads all of its bytes, the fetch
    # counter half of them
    assert abs(float(kv["write_scale"]) - 1.0) < 0.02
    assert abs(float(kv["fetch_scale"]) - 2.0) < 0.02


def test_traffic_reported_only_for_the_measured_source(monkeypatch, tmp_path):
    kv = _traffic_fields()
    if kv.get("source_sha256_16") == bench.kernel_source_hash():
        assert bench.read_traffic() == float(kv["l2_fabric_bytes_per_launch"])
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.read_traffic() is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.txt"))
    assert bench.read_traffic() is None


@pytest.mark.parametrize("n", [1, 2])
def test_ramp_replays_until_the_time_has_passed(monkeypatch, n):
    """The clock ramp replays at least once and stops once the wall time is
    spent (a stand-in graph and synchronise, no device)."""
    import types
    calls = []
    fake_torch = types.SimpleNamespace(cuda=types.SimpleNamespace(synchronize=lambda: None))
    monkeypatch.setitem(sys.modules, "torch", fake_torch)
    clock = iter(range(100))
    monkeypatch.setattr(bench.time, "perf_counter", lambda: float(next(clock)))
    graph = types.SimpleNamespace(replay=lambda: calls.append(1))
    got = bench.ramp(graph, float(n))
    assert got == len(calls) == n
    assert bench.ramp(graph, 0.0) == 1


def test_source_hash_ignores_comments_only(monkeypatch, tmp_path):
    """The traffic summary stays valid across comment edits, not code edits."""
    def digest(text):
        (tmp_path / "k.hip").write_text(text)
        monkeypatch.setattr(bench, "ROOT", str(tmp_path))
        monkeypatch.setattr(bench, "KERNEL_SOURCES", ["k.hip"])
        return bench.kernel_source_hash()
    base = digest("int f(int x) {\n  return x + 1;\n}\n")
    assert digest("// about f\nint f(int x) {  /* one more */\n\n  return x + 1;  // done\n}\n") == base
    assert digest("int f(int x) {\n  return x + 2;\n}\n") != base
