"""The CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer: a C
driver (tests/sanitize_driver.c) calls every oracle entry point in one
process built with -fsanitize=address,undefined; it must run clean and give
the same checksums as the ordinary optimised build."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRCS = [os.path.join(ROOT, "oracle", f) for f in
        ("jatam_oracle.c", "jatam_ga_oracle.c", "jatam_roulette_oracle.c")]
DRIVER = os.path.join(ROOT, "tests", "sanitize_driver.c")


def build_and_run(tmp_path, flags, name):
    exe = str(tmp_path / name)
    cmd = ["gcc", "-std=c11", "-D_GNU_SOURCE", "-pthread", "-Wall", "-Wextra", "-Werror"] + \
        flags + ["-o", exe, DRIVER] + SRCS + ["-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    return res


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not installed")
def test_oracle_is_clean_under_asan_and_ubsan(tmp_path):
    plain = build_and_run(tmp_path, ["-O2"], "driver")
    assert plain.returncode == 0, plain.stderr
    san = build_and_run(tmp_path, ["-O1", "-g", "-fno-omit-frame-pointer",
                                   "-fsanitize=address,undefined",
                                   "-fno-sanitize-recover=undefined"], "driver_san")
    assert san.returncode == 0, san.stderr[-4000:]
    assert "runtime error" not in san.stderr, san.stderr[-4000:]
    assert san.stdout == plain.stdout
