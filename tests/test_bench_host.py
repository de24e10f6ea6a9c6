"""Host-side pieces of bench.py: the profiled-traffic gate and the CLI's
refusal of more than one GPU (no GPU needed)."""
import hashlib
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _profile(tmp_path, sources, sha, traffic=123456):
    p = tmp_path / "prof.md"
    p.write_text(f"# title\n\nsources: {' '.join(sources)}\nsource_sha256: {sha}\n"
                 f"traffic_bytes_per_launch: {traffic}\n")
    return str(p)


def test_traffic_reported_while_sources_match(tmp_path):
    src = tmp_path / "k.hip"
    src.write_text("kernel v1\n")
    rel = os.path.relpath(src, ROOT)
    sha = hashlib.sha256(src.read_bytes()).hexdigest()
    assert bench.profiled_traffic(_profile(tmp_path, [rel], sha)) == 123456
    src.write_text("kernel v2\n")  # the kernel changed after profiling
    assert bench.profiled_traffic(_profile(tmp_path, [rel], sha)) is None


def test_traffic_none_for_missing_or_malformed(tmp_path):
    assert bench.profiled_traffic(str(tmp_path / "absent.md")) is None
    p = tmp_path / "bad.md"
    p.write_text("sources: a\n")
    assert bench.profiled_traffic(str(p)) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stdout


def test_single_leg_option_is_checked():
    """--leg accepts only the legs it can run alone; anything else is a
    usage error before any GPU work."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--leg", "nonsense"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "powerlaw" in r.stderr and "trsv" in r.stderr
