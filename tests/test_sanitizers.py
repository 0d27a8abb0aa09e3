"""AddressSanitizer + UBSan run of the host C code the tests rely on (the
graph generator and the CPU oracle), built with gcc on the CPU.  The driver
(tests/native/sanitize_driver.c) exercises every exported routine on small
graphs and their edge cases; any sanitizer report fails the run."""
import os
import shutil
import subprocess

import pytest

import graphgen
import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


def _build_and_run(tmp_path, extra=()):
    exe = str(tmp_path / "sanitize_driver")
    srcs = [os.path.join(HERE, "native", "sanitize_driver.c"), graphgen._SRC, oracle._SRC]
    subprocess.check_call(["gcc", "-O1", "-g", "-std=gnu11", "-fopenmp",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-fno-omit-frame-pointer", *extra, "-o", exe] + srcs + ["-lm"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="4")
    return subprocess.run([exe], env=env, capture_output=True, text=True, timeout=300)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_host_c_under_asan_ubsan(tmp_path):
    p = _build_and_run(tmp_path)
    assert p.returncode == 0, p.stdout + p.stderr
    assert "runtime error" not in p.stderr and "AddressSanitizer" not in p.stderr, p.stderr


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_sanitizer_is_active(tmp_path):
    # the same build with a planted heap overflow must be stopped
    p = _build_and_run(tmp_path, ("-DSANITIZER_SELF_TEST",))
    assert p.returncode != 0, p.stderr[-2000:]
    assert "heap-buffer-overflow" in p.stderr or "runtime error" in p.stderr, p.stderr[-2000:]
