"""The rule that decides whether a batched-run schedule read from the tuning
cache may run a plan (csrc/spd_sched.h), compiled on its own with the host
compiler and checked case by case: the cache key holds no beam shapes, so a
grid schedule (one work-group per tile) tuned on small beams must be refused
for beams whose tiles do not fit one launch."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1611_09704_amd", "csrc")
MAX_ITEMS = 0xFFFFFFFF

CASES = [
    # X, win, wgs_per_cu, grab, has_win, tiles, waves, expected
    (8, 0, 0, 1, False, 1000, 4, 1),                  # grid launch that fits
    (8, 0, 0, 1, False, MAX_ITEMS // 256 + 1, 4, 0),   # grid launch one tile too many
    (8, 0, 0, 1, False, MAX_ITEMS // 256, 4, 1),       # exactly the largest grid
    (8, 0, 4, 8, False, 10 ** 9, 4, 1),                # persistent: any tile count
    (4, 0, 2, 1, False, 10 ** 9, 4, 1),
    (8, 1, 0, 1, True, 1000, 4, 1),                    # register-window grid
    (8, 1, 0, 1, False, 1000, 4, 0),                   # ... not built for this plan
    (8, 1, 4, 1, True, 1000, 4, 0),                    # ... has no persistent variant
    (4, 1, 0, 1, True, 1000, 4, 0),                    # ... runs 8 outputs per lane only
    (8, 1, 0, 1, True, MAX_ITEMS // 256 + 1, 4, 0),    # ... too many tiles for one launch
    (6, 0, 0, 1, False, 10, 4, 0),                     # fields out of range
    (8, 0, -1, 1, False, 10, 4, 0),
    (8, 0, 4, 0, False, 10, 4, 0),
]


@pytest.fixture(scope="module")
def rule_binary(tmp_path_factory):
    d = tmp_path_factory.mktemp("sched")
    src = d / "rule.cpp"
    src.write_text('#include <cstdio>\n#include <cstdlib>\n#include "spd_sched.h"\n'
                   "int main(int argc, char** argv) {\n"
                   "  if (argc != 9) return 2;\n"
                   "  long long v[8];\n"
                   "  for (int i = 0; i < 8; ++i) v[i] = std::strtoll(argv[i + 1], nullptr, 10);\n"
                   "  std::printf(\"%d\\n\", (int)spd::schedule_usable((int)v[0], (int)v[1], (int)v[2], (int)v[3],\n"
                   "      v[4] != 0, (int64_t)v[5], (int)v[6], (uint64_t)v[7]));\n"
                   "  return 0;\n}\n")
    exe = d / "rule"
    subprocess.run(["g++", "-std=c++17", "-O1", "-I" + CSRC, str(src), "-o", str(exe)], check=True)
    return str(exe)


@pytest.mark.parametrize("case", CASES)
def test_cached_schedule_rule(rule_binary, case):
    *args, expected = case
    out = subprocess.run([rule_binary] + [str(int(a)) for a in args] + [str(MAX_ITEMS)],
                         check=True, capture_output=True, text=True).stdout.strip()
    assert int(out) == expected, case
