"""Host logic of bench.py: the one-GPU guard and the use of the committed HBM counters."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and "--gpus 2" in r.stderr
    assert r.stdout == ""


def test_traffic_is_used_only_for_the_kernel_source_it_was_measured_on(monkeypatch):
    d = os.path.join(ROOT, "profiles")
    files = [f for f in os.listdir(d) if f.startswith("traffic_stream_collide_")]
    assert files, "no committed HBM counter summary"
    for f in files:
        rec = json.load(open(os.path.join(d, f)))
        wl, st, lay = rec["workload"], rec["storage"], rec["layout"]
        assert f == f"traffic_stream_collide_{wl}_{st}_{lay}.json"
        # read + written bytes, and the summary beside it names the same source hash
        assert rec["bytes_per_launch"] == rec["bytes_read"] + rec["bytes_written"]
        md = open(os.path.join(d, f"stream_collide_{wl}_{st}_{lay}.md")).read()
        assert f"kernel source hash: {rec['kernel_source_hash']}" in md
        monkeypatch.setattr(bench, "kernel_source_hash", lambda h=rec["kernel_source_hash"]: h)
        assert bench.measured_traffic(wl, st, lay) == rec["bytes_per_launch"]
        other = "compact" if lay == "dense" else "dense"
        if not os.path.exists(os.path.join(d, f"traffic_stream_collide_{wl}_{st}_{other}.json")):
            assert bench.measured_traffic(wl, st, other) is None
        monkeypatch.setattr(bench, "kernel_source_hash", lambda: "changed")
        assert bench.measured_traffic(wl, st, lay) is None
    assert bench.measured_traffic("no_such_workload", "f32", "dense") is None

