"""AddressSanitizer / UndefinedBehaviorSanitizer builds of the host side of
libebic (evolution steps, screened pools, stateful runs and checkpoints,
driven by a fake evaluator) and of the C oracle, run on the CPU."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1801_03039_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
       "-fno-omit-frame-pointer", "-g", "-O1"]

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")


def _run(exe):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    return r.stdout


def test_host_side_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_driver")
    cmd = (["g++", "-std=c++17"] + SAN +
           ["-I", os.path.join(ROOT, "include"), "-I", CSRC,
            os.path.join(HERE, "sanitize", "host_driver.cpp"),
            os.path.join(CSRC, "ebic_evolve.cpp"), os.path.join(CSRC, "ebic_checkpoint.cpp"),
            "-o", exe, "-lpthread"])
    subprocess.run(cmd, check=True, capture_output=True, timeout=600)
    assert "host driver ok" in _run(exe)


def test_host_side_under_thread_sanitizer(tmp_path):
    # data races in the host threads of screened runs (persistent helper
    # threads drawing the pool's shares, hashing the pool in parallel)
    exe = str(tmp_path / "host_driver_tsan")
    cmd = (["g++", "-std=c++17", "-fsanitize=thread", "-g", "-O1",
            "-I", os.path.join(ROOT, "include"), "-I", CSRC,
            os.path.join(HERE, "sanitize", "host_driver.cpp"),
            os.path.join(CSRC, "ebic_evolve.cpp"), os.path.join(CSRC, "ebic_checkpoint.cpp"),
            "-o", exe, "-lpthread"])
    subprocess.run(cmd, check=True, capture_output=True, timeout=600)
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1:second_deadlock_stack=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "host driver ok" in r.stdout
    assert "WARNING: ThreadSanitizer" not in r.stderr, r.stderr[-4000:]


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    cmd = (["gcc", "-std=c11", "-fopenmp"] + SAN +
           [os.path.join(HERE, "sanitize", "oracle_driver.c"),
            os.path.join(ROOT, "oracle", "ebic_oracle.c"), "-o", exe, "-lm"])
    subprocess.run(cmd, check=True, capture_output=True, timeout=600)
    assert "oracle driver ok" in _run(exe)
