"""Host logic of bench.py (no GPU): the one-GPU guard and the lookup of the
committed rocprofv3 traffic summary."""
import hashlib
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       cwd=ROOT, timeout=300)
    assert r.returncode != 0
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_profile_traffic_lookup(tmp_path, monkeypatch):
    # a summary is used only while the kernel sources it was taken on are
    # unchanged (sha256 of tip.hip + dev_common.h)
    csrc = tmp_path / "paper_2110_12511_amd" / "csrc"
    csrc.mkdir(parents=True)
    (csrc / "tip.hip").write_bytes(b"kernel a")
    (csrc / "dev_common.h").write_bytes(b"helpers")
    prof = tmp_path / "profiles"
    prof.mkdir()
    sha = hashlib.sha256(b"kernel a" + b"helpers").hexdigest()
    (prof / "k_tip_peel_tiled__wl.md").write_text(
        f"```\nkernel: k_tip_peel_tiled\ntraffic_bytes_per_launch: 123456\nsource_sha256: {sha}\n```\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.profile_traffic("tip_tiled", "wl") == 123456
    assert bench.profile_traffic("tip_tiled", "other") is None
    assert bench.profile_traffic("wing_cd", "wl") is None
    (csrc / "tip.hip").write_bytes(b"kernel b")
    assert bench.profile_traffic("tip_tiled", "wl") is None


def test_committed_summary_is_well_formed():
    path = os.path.join(ROOT, "profiles", "k_tip_peel_hrange__tip_u_cl_5m_1m_100m.md")
    text = open(path).read()
    assert "traffic_bytes_per_launch:" in text and "source_sha256:" in text
    assert "rocprofv3 --kernel-trace --stats" in text and "--pmc FETCH_SIZE" in text and "--pmc WRITE_SIZE" in text
    # the summary was taken on the current kernel sources
    import bench

    assert bench.profile_traffic("tip_hrange", "tip_u_cl_5m_1m_100m") is not None
