"""The C oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc, host code only) and driven through every entry point: no memory error,
no undefined behaviour, no leak, and the same output checksum as the plain
optimised build.  A copy of the oracle with an out-of-bounds write planted in
the systematic subsets shows that the sanitized build reports such a
mistake."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE_DIR = os.path.join(os.path.dirname(HERE), "oracle")
DRIVER = os.path.join(HERE, "oracle_sanitize_driver.c")
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc is not installed")


def _build(out, flags, include=ORACLE_DIR):
    cmd = ["gcc", "-std=c11", "-fno-fast-math", "-Wall", "-Wextra", *flags, "-I", include, DRIVER, "-o", out, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=120)
    if r.returncode != 0 and "-fsanitize=address,undefined" in flags and "asan" in r.stderr:
        pytest.skip("gcc has no sanitizer runtime here: " + r.stderr[-200:])
    assert r.returncode == 0, r.stderr
    return out


def _run(exe):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    return subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)


def test_oracle_is_clean_under_sanitizers(tmp_path):
    plain = _run(_build(str(tmp_path / "plain"), ["-O2"]))
    san = _run(_build(str(tmp_path / "san"), SAN))
    assert plain.returncode == 0, plain.stderr[-2000:]
    assert san.returncode == 0, san.stderr[-4000:]
    assert "runtime error" not in san.stderr and "Sanitizer" not in san.stderr, san.stderr[-4000:]
    assert plain.stdout.startswith("checksum ")
    assert san.stdout == plain.stdout


def test_sanitized_build_reports_a_planted_overflow(tmp_path):
    src = open(os.path.join(ORACLE_DIR, "pns_oracle.c")).read()
    anchor = "for (int32_t t = 0; t < n; ++t) member[(start + t) % N] = 1;"
    assert anchor in src
    (tmp_path / "pns_oracle.c").write_text(src.replace(anchor, "for (int32_t t = 0; t < n; ++t) member[start + t] = 1;"))
    r = _run(_build(str(tmp_path / "mutant"), SAN, include=str(tmp_path)))
    assert r.returncode != 0
    assert "heap-buffer-overflow" in r.stderr
