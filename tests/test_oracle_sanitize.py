"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (gcc,
host code only) runs every exported routine on small inputs and invalid
arguments (tests/oracle_sanitize_driver.c).  A second build of a copy of the
oracle with one out-of-bounds write planted in it must be caught, so that a
silent sanitizer setup cannot pass."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DRIVER = os.path.join(ROOT, "tests", "oracle_sanitize_driver.c")
ORACLE = os.path.join(ROOT, "oracle", "gabor_oracle.c")
FLAGS = ["-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
         "-fno-sanitize-recover=all"]


def build(tmp_path, oracle_src, name):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / name)
    r = subprocess.run([gcc] + FLAGS + [DRIVER, oracle_src, "-lm", "-o", exe], capture_output=True, text=True)
    if r.returncode != 0 and "asan" in r.stderr.lower():
        pytest.skip("sanitizer runtime not available: " + r.stderr.strip()[:200])
    assert r.returncode == 0, r.stderr
    return exe


def run(exe):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    return subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)


def test_oracle_is_clean_under_sanitizers(tmp_path):
    r = run(build(tmp_path, ORACLE, "oracle_sanitize"))
    assert r.returncode == 0, r.stdout + r.stderr
    assert "oracle sanitizer run: ok" in r.stdout


def test_sanitizers_catch_a_planted_overflow(tmp_path):
    with open(ORACLE) as fh:
        src = fh.read()
    clean = "for (int t = 0; t < 2 * R + 1; ++t) taps[t] /= sum;"
    assert clean in src
    planted = str(tmp_path / "gabor_oracle_planted.c")
    with open(planted, "w") as fh:
        fh.write(src.replace(clean, "for (int t = 0; t <= 2 * R + 1; ++t) taps[t] /= sum;"))
    r = run(build(tmp_path, planted, "oracle_planted"))
    assert r.returncode != 0
    assert "AddressSanitizer" in r.stderr
