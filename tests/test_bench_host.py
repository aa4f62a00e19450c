"""Host-side parts of bench.py that need no GPU: the one-GPU refusal, the
lookup of measured HBM traffic (reported only while the interaction
kernels' sources still hash to the value stored with the counters) and the
comment stripping that hash is taken over."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2, r.stderr[-2000:]
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def _stored():
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as fh:
        return json.load(fh)


def test_traffic_only_for_the_sources_it_was_taken_on(monkeypatch):
    d = _stored()
    wl = next(iter(d["workloads"]))
    kern = next(iter(d["workloads"][wl]))
    stored = d["workloads"][wl][kern]
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: stored["source_hash"])
    b = bench.measured_traffic(kern, wl)
    assert b == stored["bytes_per_launch"] and b > 0
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.measured_traffic(kern, wl) is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: stored["source_hash"])
    assert bench.measured_traffic(kern, "no_such_workload") is None
    assert bench.measured_traffic("no_such_kernel", wl) is None


def test_hash_ignores_comments_not_code():
    a = "int a; // the count\n/* block\n comment */\nint b;\n\n"
    b = "int a;\nint b;"
    assert bench._strip_comments(a, False) == bench._strip_comments(b, False)
    assert bench._strip_comments("int a;\nint c;", False) != bench._strip_comments(b, False)
    assert bench._strip_comments("x = 1  # note\n\ny = 2\n", True) == "x = 1\ny = 2"


@pytest.mark.parametrize("f", bench.KERNEL_SOURCES)
def test_hashed_sources_exist(f):
    assert os.path.isfile(os.path.join(ROOT, f))
