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
    """A counter record is used only for the launch size it was taken at
    and only while its recorded source hash equals the current sources'."""
    sys.path.insert(0, ROOT)
    import bench
    with open(os.path.join(ROOT, "profiles", "kk_front_kk16qam_2e22_b64_traffic.json")) as f:
        rec = json.load(f)
    fake = tmp_path / "profiles"
    fake.mkdir()
    os.symlink(os.path.join(ROOT, "paper_2010_14333_amd"), tmp_path / "paper_2010_14333_amd")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    rec["source_sha256"] = bench.kernel_source_hash()
    (fake / "kk_front_kk16qam_2e22_b64_traffic.json").write_text(json.dumps(rec))
    t = bench.front_traffic(64)
    assert t is not None and t["bytes_per_launch"] == rec["bytes_per_launch"]
    assert bench.front_traffic(16) is None   # recorded for 64-buffer launches only
    rec["source_sha256"] = "0" * 64
    (fake / "kk_front_kk16qam_2e22_b64_traffic.json").write_text(json.dumps(rec))
    assert bench.front_traffic(64) is None


def test_traffic_figure_survives_comments_not_code(tmp_path, monkeypatch):
    """The counters belong to the code: a copy of the sources with an added
    comment keeps the figure, one with a changed constant turns it off."""
    import shutil
    sys.path.insert(0, ROOT)
    import bench
    (tmp_path / "profiles").mkdir()
    with open(os.path.join(ROOT, "profiles", "kk_front_kk16qam_2e22_b64_traffic.json")) as f:
        rec = json.load(f)
    rec["source_sha256"] = bench.kernel_source_hash()
    (tmp_path / "profiles" / "kk_front_kk16qam_2e22_b64_traffic.json").write_text(json.dumps(rec))
    src = tmp_path / "paper_2010_14333_amd" / "csrc"
    src.mkdir(parents=True)
    for name in bench.KERNEL_SOURCES:
        shutil.copy(os.path.join(ROOT, "paper_2010_14333_amd", "csrc", name), src / name)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    kk = src / "kk.hip"
    text = kk.read_text()
    kk.write_text("// a note for readers\n" + text.replace("\n\n", "\n\n/* and another */\n", 1))
    assert bench.front_traffic(64) is not None
    assert "constexpr int RG = fpad(1024);" in text
    kk.write_text(text.replace("constexpr int RG = fpad(1024);", "constexpr int RG = fpad(1024) + 2;"))
    assert bench.front_traffic(64) is None
