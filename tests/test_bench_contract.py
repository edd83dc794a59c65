"""Host-side checks of bench.py: the recorded counter traffic is tied to the
kernel sources and to a committed profile summary, and a request for more than
one GPU is refused with a message."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


@pytest.mark.parametrize("key", sorted(bench.TRAFFIC_RECORD))
def test_traffic_record_names_its_sources_and_summary(key):
    rec = bench.TRAFFIC_RECORD[key]
    assert rec["kernel"] in bench.KERNEL_SOURCES
    for f in bench.KERNEL_SOURCES[rec["kernel"]]:
        assert os.path.exists(os.path.join(ROOT, f)), f
    summary = os.path.join(ROOT, rec["summary"])
    assert os.path.exists(summary), summary
    text = open(summary).read()
    # the summary states the counter values and the source hash they belong to
    assert rec["sha256_prefix"] in text
    assert ("%.1f" % rec["fetch_kib"]) in text and ("%.1f" % rec["write_kib"]) in text
    assert rec["fetch_scale"] > 0 and rec["write_scale"] > 0


def test_traffic_is_null_once_a_source_changes(monkeypatch):
    key = sorted(bench.TRAFFIC_RECORD)[0]
    rec = dict(bench.TRAFFIC_RECORD[key], sha256_prefix="0" * 16)
    monkeypatch.setitem(bench.TRAFFIC_RECORD, key, rec)
    assert bench.recorded_traffic(*key) is None
    assert bench.recorded_traffic("no-such-workload", "fp32") is None


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert p.returncode != 0
    assert "one GPU" in p.stderr
    assert p.stdout.strip() == ""
