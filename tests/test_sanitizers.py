"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* the library's host-side input checks (paper_1506_04383_amd/csrc/validate.cpp:
  graphs, general stress sets, autotuner records) built with g++ and driven by
  tests/sanitize/driver_validate.cpp on valid, malformed and 40,000 random
  arrays of the documented sizes;
* the FP64 oracle (oracle/mm_oracle.c) built with gcc and driven by
  tests/sanitize/driver_oracle.c through every entry point on small graphs
  and point sets, including two vertices, a star and coincident points.

A sanitizer report aborts the driver (-fno-sanitize-recover=all), so the
test passes only when both drivers exit 0 with no report.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-g", "-O1", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


def _run(cmd, env=None):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300, env=env)
    out = r.stdout + r.stderr
    return r.returncode, out


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_checks_under_sanitizers(tmp_path):
    exe = str(tmp_path / "driver_validate")
    rc, out = _run(["g++", "-std=c++17", *SAN, "-I", os.path.join(ROOT, "paper_1506_04383_amd", "csrc"),
                    os.path.join(ROOT, "tests", "sanitize", "driver_validate.cpp"),
                    os.path.join(ROOT, "paper_1506_04383_amd", "csrc", "validate.cpp"), "-o", exe])
    assert rc == 0, out
    rc, out = _run([exe])
    print(out)
    assert rc == 0 and "runtime error" not in out and "AddressSanitizer" not in out, out


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "driver_oracle")
    rc, out = _run(["gcc", "-std=c11", *SAN, "-fopenmp", "-I", os.path.join(ROOT, "oracle"),
                    os.path.join(ROOT, "oracle", "mm_oracle.c"),
                    os.path.join(ROOT, "tests", "sanitize", "driver_oracle.c"), "-lm", "-o", exe])
    assert rc == 0, out
    rc, out = _run([exe], env=dict(os.environ, OMP_NUM_THREADS="2"))
    print(out)
    assert rc == 0 and "runtime error" not in out and "AddressSanitizer" not in out, out
