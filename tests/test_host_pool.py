"""The host worker pool of the build's host phase (csrc/hostpool.hpp), checked
natively: a stress program built with g++ under ThreadSanitizer (host code
only) runs concurrent and nested loops and verifies that every index is
visited exactly once; ThreadSanitizer fails the run on a data race."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
@pytest.mark.parametrize("sanitize", [False, True])
def test_host_pool_visits_every_index_once(tmp_path, sanitize):
    src = os.path.join(HERE, "native", "hostpool_check.cpp")
    exe = str(tmp_path / "hostpool_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-pthread", src, "-o", exe]
    if sanitize:
        cmd.insert(1, "-fsanitize=thread")
    r = subprocess.run(cmd, capture_output=True, text=True)
    if sanitize and r.returncode != 0 and "sanitize" in r.stderr:
        pytest.skip("ThreadSanitizer is not available")
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66")
    out = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "errors 0" in out.stdout
