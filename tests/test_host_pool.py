"""The compaction engine's host thread pool under ThreadSanitizer (no GPU needed)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_pool_runs_every_item_once_without_races(tmp_path):
    exe = tmp_path / "pool_stress"
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=thread", "-pthread",
                           "-I", os.path.join(ROOT, "paper_2208_14935_amd", "csrc"),
                           os.path.join(ROOT, "tests", "cpp", "pool_stress.cpp"), "-o", str(exe)])
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ok" in r.stdout
