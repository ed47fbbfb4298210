"""The serving form's admission and deadline policy (csrc/spd_admit.h, the
code the server's worker thread runs), checked on the host with a fake clock
and a fake executor: per-beam order, at most slots_per_beam chunks of a beam
and at most the pool's buffers on the device, no admissible request skipped
while a buffer is free, no starvation under backpressure and bursts, a
failed launch dropping its request and returning its buffer, and deadlines."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_1611_09704_amd", "csrc")


def test_admission_policy_with_fake_clock(tmp_path):
    exe = str(tmp_path / "serve_policy_check")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-Wall", "-Werror", "-I", CSRC,
                           os.path.join(HERE, "serve_policy_check.cpp"), "-o", exe])
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0 and out.stdout.strip().endswith("ok"), out.stdout + out.stderr
