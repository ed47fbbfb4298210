"""Host code under the address and undefined-behaviour sanitizers: the C
oracle (driven over every scope, sigma mode and edge shape with exactly
sized buffers) and the serving admission policy.  CPU only; the GPU library
itself is checked for bounds by the canary tests."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = ["-fsanitize=" + s for s in ("address", "undefined")] + ["-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def _build_and_run(cmd, exe):
    subprocess.check_call(cmd + ["-o", exe])
    out = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=ENV)
    assert out.returncode == 0 and out.stdout.strip().endswith("ok"), out.stdout + out.stderr


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_sanitizers(tmp_path):
    _build_and_run(["gcc", "-std=c11", "-O1", "-g", "-fopenmp"] + SAN +
                   [os.path.join(ROOT, "oracle", "spd_oracle.c"), os.path.join(HERE, "oracle_sanitize_driver.c"),
                    "-lm"], str(tmp_path / "oracle_san"))


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not found")
def test_serve_policy_under_sanitizers(tmp_path):
    _build_and_run(["g++", "-std=c++17", "-O1", "-g"] + SAN +
                   ["-I", os.path.join(ROOT, "paper_1611_09704_amd", "csrc"),
                    os.path.join(HERE, "serve_policy_check.cpp")], str(tmp_path / "policy_san"))
