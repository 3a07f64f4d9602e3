"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

oracle.c is built with -fsanitize=address,undefined (host code only; nothing
here touches a GPU) and the pin suite runs against that build in a
subprocess, with the ASan runtime preloaded into the interpreter so that the
arrays numpy hands to the oracle sit in sanitizer-checked heap memory.  A
second case plants an out-of-bounds read in a copy of the oracle and
requires the sanitizer run to report it, so a silent sanitizer cannot pass
the first case."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")


def _runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def _build(src_text, out_dir):
    src = os.path.join(out_dir, "oracle.c")
    with open(src, "w") as fh:
        fh.write(src_text)
    with open(os.path.join(out_dir, "oracle.h"), "w") as fh:
        fh.write(open(os.path.join(ROOT, "oracle", "oracle.h")).read())
    so = os.path.join(out_dir, "liboracle_san.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", "-fopenmp",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                           "-fno-omit-frame-pointer", src, "-o", so, "-lm"])
    return so


def _run_pins(so, log_dir, select=None):
    """Run the pin suite against `so`; returns the process and the text of
    the sanitizer reports (written to files: pytest's output capture would
    swallow a report printed by a process that the sanitizer ends)."""
    asan = _runtime("libasan.so")
    pre = os.environ.get("LD_PRELOAD", "")
    log = os.path.join(log_dir, "san")
    env = dict(os.environ, PILOT_ORACLE_LIB_OVERRIDE=so, LD_PRELOAD=(asan + (" " + pre if pre else "")),
               ASAN_OPTIONS=f"detect_leaks=0:abort_on_error=0:log_path={log}",
               UBSAN_OPTIONS=f"halt_on_error=1:print_stacktrace=1:log_path={log}")
    cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
           os.path.join(ROOT, "tests", "test_oracle_pins.py")]
    if select:
        cmd += ["-k", select]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    reports = "".join(open(os.path.join(log_dir, f)).read() for f in sorted(os.listdir(log_dir))
                      if f.startswith("san"))
    return r, reports


pytestmark = pytest.mark.skipif(_runtime("libasan.so") is None, reason="gcc's ASan runtime is not installed")


def test_pin_suite_is_clean_under_asan_and_ubsan(tmp_path):
    so = _build(open(SRC).read(), str(tmp_path))
    r, reports = _run_pins(so, str(tmp_path))
    assert r.returncode == 0, (r.stdout + r.stderr)[-3000:] + reports[:3000]
    assert reports == "", reports[:3000]


def test_sanitizer_reports_a_planted_out_of_bounds_read(tmp_path):
    old = "val[c] = (1.0 - ax) * (1.0 - ay) * f00[c]"
    src = open(SRC).read()
    assert src.count(old) == 1
    so = _build(src.replace(old, "val[c] = (1.0 - ax) * (1.0 - ay) * f00[c + 2 * C * W * H]"), str(tmp_path))
    r, reports = _run_pins(so, str(tmp_path), select="bilinear")
    assert r.returncode != 0
    assert "ERROR: AddressSanitizer" in reports and "orc_bilinear" in reports, reports[:2000]
