"""The oracle's C code under AddressSanitizer + UndefinedBehaviorSanitizer
(leaks included) and under ThreadSanitizer (its solver runs runs on worker
threads): tests/oracle_sanitize_driver.c drives every instance kind, both
schedules, phased, synchronous and damped updates, the per-level records and
their replay.  A report from either sanitizer fails the test."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
DRIVER = os.path.join(HERE, "oracle_sanitize_driver.c")

BUILDS = {
    "address+undefined": (["-fsanitize=address,undefined", "-fno-sanitize-recover=all"],
                          {"ASAN_OPTIONS": "verify_asan_link_order=0:detect_leaks=1:halt_on_error=1",
                           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}),
    "thread": (["-fsanitize=thread"], {"TSAN_OPTIONS": "halt_on_error=1"}),
}


@pytest.mark.parametrize("name", list(BUILDS))
def test_oracle_under_sanitizer(name, tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    flags, env = BUILDS[name]
    exe = str(tmp_path / "driver")
    build = subprocess.run(["gcc", "-std=c11", "-O1", "-g", "-ffp-contract=off", "-pthread", *flags, DRIVER, "-lm",
                            "-o", exe], capture_output=True, text=True)
    if build.returncode != 0 and "sanitize" in build.stderr:
        pytest.skip("sanitizer runtime not available: " + build.stderr[-200:])
    assert build.returncode == 0, build.stderr
    run = subprocess.run([exe], capture_output=True, text=True, timeout=300, env={**os.environ, **env})
    assert run.returncode == 0 and run.stdout.rstrip().endswith("OK"), run.stdout + run.stderr
