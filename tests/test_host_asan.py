"""Host code under AddressSanitizer + UndefinedBehaviorSanitizer (no GPU needed): the input
generator at vertex counts that are not powers of two, and the runtime's hub sorting."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None, reason="gcc/g++ not available")
def test_generator_and_hub_sort_are_clean_under_asan_ubsan(tmp_path):
    san = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
    gobj = tmp_path / "gen.o"
    subprocess.check_call(["gcc", *san, "-c", os.path.join(ROOT, "gen", "gen.c"), "-o", str(gobj)])
    exe = tmp_path / "host_asan"
    csrc = os.path.join(ROOT, "paper_2208_14935_amd", "csrc")
    subprocess.check_call(["g++", "-std=c++17", *san, "-pthread", "-I", csrc,
                           os.path.join(ROOT, "tests", "cpp", "host_asan.cpp"), os.path.join(csrc, "hubsort.cpp"),
                           str(gobj), "-o", str(exe)])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-4000:]
    assert "ok" in r.stdout
