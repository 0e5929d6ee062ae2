"""Host-side race test of the ring drain's copy pool (copy_pool.h), built with
g++ alone: each of many back-to-back runs must run every chunk exactly once,
and a thread-sanitizer build must report no race (a late worker touching a
finished run's bounds or function object)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "copy_pool_stress.cpp")


def _build(tmp_path, extra):
    exe = str(tmp_path / ("stress" + ("_tsan" if extra else "")))
    subprocess.check_call(["g++", "-O1", "-g", "-std=c++17", "-pthread"] + extra + [SRC, "-o", exe])
    return exe


def test_copy_pool_every_chunk_once(tmp_path):
    exe = _build(tmp_path, [])
    out = subprocess.run([exe, "50000", "6"], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.startswith("ok")


def test_copy_pool_no_race_under_tsan(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("no g++")
    try:
        exe = _build(tmp_path, ["-fsanitize=thread"])
    except subprocess.CalledProcessError:
        pytest.skip("thread sanitizer not available")
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1")
    out = subprocess.run([exe, "5000", "4"], capture_output=True, text=True, timeout=600, env=env)
    assert out.returncode == 0, out.stderr[-4000:]
    assert "ThreadSanitizer" not in out.stderr
