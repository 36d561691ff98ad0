"""Host-side checks of bench.py (no device): the multi-GPU request is
refused with a message, the output line is strict JSON, and the traffic
counters are reported only for the kernel sources they were taken with."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_strict_json():
    import bench
    line = json.dumps(bench.strict_json({"a": float("nan"), "b": [1.0, float("inf")], "c": {"d": -float("inf")}}),
                      allow_nan=False)
    assert json.loads(line) == {"a": None, "b": [1.0, None], "c": {"d": None}}


def test_traffic_bound_to_sources(monkeypatch):
    """The counters' traffic is reported only for the kernel sources, tile
    shape and kernel they were taken with."""
    import hashlib

    import bench
    h = hashlib.sha256()
    for f in bench.TRAFFIC_SOURCES:
        with open(os.path.join(bench.ROOT, f), "rb") as fh:
            h.update(fh.read())
    current = h.hexdigest()[:16]
    tile = bench.TRAFFIC["tile"]
    monkeypatch.setitem(bench.TRAFFIC, "sha", current)
    t = bench.measured_traffic("face_xy", tile)
    assert t is not None and t > 0
    assert bench.measured_traffic("face_xy", tile + 1) is None
    assert bench.measured_traffic("no_such_kernel", tile) is None
    monkeypatch.setitem(bench.TRAFFIC, "sha", "0" * 16)
    assert bench.measured_traffic("face_xy", tile) is None
