"""The library's host runtime under AddressSanitizer and UndefinedBehaviorSanitizer.

pilot_runtime.cpp (argument validation, planning, workspace layout, graph
cache, serving slots) is compiled by g++ with the sanitizers and linked with
the normal build's HIP objects (paper_2606_31098_amd/build_host_sanitized.py).
On the CPU only the device-free entry points run, so the ABI checks run here
against that copy; the GPU suite runs against it the same way on a GPU
(PILOT_LIB_OVERRIDE, with the same preloads).  A second case plants an
out-of-bounds read in a copy of the runtime and requires the sanitizer to
report it, so a silent sanitizer cannot pass the first case."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
RT = os.path.join(ROOT, "paper_2606_31098_amd", "csrc", "pilot_runtime.cpp")


def _runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def _hip_objects_present():
    from paper_2606_31098_amd import build as B
    return all(os.path.exists(os.path.join(B.OBJ, os.path.basename(s) + ".o"))
               for s in B.sources() if s.endswith(".hip"))


pytestmark = pytest.mark.skipif(_runtime("libasan.so") is None or not _hip_objects_present(),
                                reason="gcc's ASan runtime or the library's build objects are missing")


def _run_abi_tests(so, log_dir, select=None):
    pre = os.environ.get("LD_PRELOAD", "")
    preload = " ".join(p for p in (_runtime("libasan.so"), _runtime("libstdc++.so.6"), pre) if p)
    log = os.path.join(log_dir, "san")
    env = dict(os.environ, PILOT_LIB_OVERRIDE=so, LD_PRELOAD=preload,
               ASAN_OPTIONS=f"detect_leaks=0:verify_asan_link_order=0:abort_on_error=0:log_path={log}",
               UBSAN_OPTIONS=f"halt_on_error=1:print_stacktrace=1:log_path={log}")
    cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
           os.path.join(ROOT, "tests", "test_abi.py")]
    if select:
        cmd += ["-k", select]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    reports = "".join(open(os.path.join(log_dir, f)).read() for f in sorted(os.listdir(log_dir))
                      if f.startswith("san"))
    return r, reports


def test_abi_checks_are_clean_under_asan_and_ubsan(tmp_path):
    from paper_2606_31098_amd.build_host_sanitized import build_host_sanitized
    so = build_host_sanitized(str(tmp_path / "lib"))
    r, reports = _run_abi_tests(so, str(tmp_path))
    assert r.returncode == 0, (r.stdout + r.stderr)[-3000:] + reports[:3000]
    assert "passed" in r.stdout and reports == "", reports[:3000]


def test_sanitizer_reports_a_planted_out_of_bounds_read(tmp_path):
    from paper_2606_31098_amd.build_host_sanitized import build_host_sanitized
    old = "    if (!name) return 0;\n    if (!strcmp(name, \"pilot_frame\")) return sizeof(pilot_frame);"
    src = open(RT).read()
    assert src.count(old) == 1
    planted = ("    if (!name) return 0;\n"
               "    { std::vector<char> v(4); volatile char c = v.data()[name[0] == 'p' ? 8 : 0]; (void)c; }\n"
               "    if (!strcmp(name, \"pilot_frame\")) return sizeof(pilot_frame);")
    bad = tmp_path / "pilot_runtime.cpp"
    bad.write_text(src.replace(old, planted))
    so = build_host_sanitized(str(tmp_path / "lib"), runtime_src=str(bad))
    r, reports = _run_abi_tests(so, str(tmp_path), select="struct_layouts")
    assert r.returncode != 0
    assert "ERROR: AddressSanitizer: heap-buffer-overflow" in reports and "pilot_sizeof" in reports, reports[:2000]
