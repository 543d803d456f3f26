"""bench.py's command-line contract that needs no GPU: more than one GPU is
refused with a message before anything touches a device, and the front
end's committed traffic figure is used only while its source hash matches."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_figure_follows_the_sources(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    t = bench.front_traffic(64)
    with open(os.path.join(ROOT, "profiles", "kk_front_kk16qam_2e22_b64_traffic.json")) as f:
        rec = json.load(f)
    assert t is not None and t["bytes_per_launch"] == rec["bytes_per_launch"]
    assert bench.front_traffic(16) is None   # recorded for 64-buffer launches only
    # a recorded hash that does not match the sources turns the figure off
    fake = tmp_path / "profiles"
    fake.mkdir()
    rec["source_sha256"] = "0" * 64
    (fake / "kk_front_kk16qam_2e22_b64_traffic.json").write_text(json.dumps(rec))
    os.symlink(os.path.join(ROOT, "paper_2010_14333_amd"), tmp_path / "paper_2010_14333_amd")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.front_traffic(64) is None
