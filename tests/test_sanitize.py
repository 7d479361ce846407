"""Sanitizer builds of host code (no GPU): the FP64 oracle under AddressSanitizer +
UndefinedBehaviorSanitizer (gcc), driven through every function and its edge cases
(tests/sanitize/oracle_driver.c).  Any sanitizer report aborts the driver."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def _run(cmd, **kw):
    res = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert res.returncode == 0, f"{' '.join(cmd)}\n{res.stdout}\n{res.stderr}"
    return res


def test_oracle_under_asan_ubsan(tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("gcc not found")
    exe = str(tmp_path / "oracle_driver")
    _run(["gcc", "-O1", "-g", "-std=c11", "-fopenmp", *SAN, "-o", exe, os.path.join(HERE, "oracle_driver.c"),
          os.path.join(ROOT, "oracle", "joseph64.c"), "-lm"])
    res = _run([exe], env={**os.environ, "OMP_NUM_THREADS": "4"})
    assert "oracle driver: ok" in res.stdout
