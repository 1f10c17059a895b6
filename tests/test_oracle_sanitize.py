"""The FP64 oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc, host code only, OpenMP off) and driven through every entry point on
small seeded inputs (oracle/sanitize_driver.c): no out-of-bounds access, use
after free, leak or undefined operation may be reported."""
import os
import shutil
import subprocess

import pytest

from conftest import ROOT

SRCS = ["sanitize_driver.c", "mf4d_oracle.c", "net_oracle.c", "crease_oracle.c", "mf4d3d_oracle.c"]


def test_oracle_under_sanitizers(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no gcc")
    exe = tmp_path / "oracle_sanitized"
    cmd = [gcc, "-O1", "-g", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-o", str(exe),
           *[os.path.join(ROOT, "oracle", f) for f in SRCS], "-lm"]
    built = subprocess.run(cmd, capture_output=True, text=True)
    assert built.returncode == 0, built.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=900)
    assert run.returncode == 0, (run.stdout + run.stderr)[-4000:]
    assert "oracle sanitizer run: ok" in run.stdout
    assert "runtime error" not in run.stderr and "ERROR: AddressSanitizer" not in run.stderr
