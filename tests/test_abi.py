"""The C-ABI library loads and exports every entry point include/pilot.h
declares, with matching struct layouts.  CPU only: no compute calls."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pilot.h")
# the in-tree library, or the build PILOT_LIB_OVERRIDE names (the host-sanitized copy)
LIB = os.environ.get("PILOT_LIB_OVERRIDE") or os.path.join(ROOT, "paper_2606_31098_amd", "libpilot.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pilot_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2606_31098_amd import build
        build.build()
    return C.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["pilot_create", "pilot_solve", "pilot_destroy", "pilot_last_error", "pilot_linearize",
                     "pilot_admit", "pilot_step", "pilot_poll"]:
        assert required in names


def test_library_exports_every_declared_function(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r" T (pilot_\w+)", out))
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing
    for n in declared_functions():
        getattr(lib, n)


def test_struct_layouts_match_binding(lib):
    from paper_2606_31098_amd import _abi as A
    L = A.load(LIB)
    assert L.pilot_abi_version() == 1
    for name, cls in [("pilot_frame", A.Frame), ("pilot_level", A.Level), ("pilot_result", A.Result),
                      ("pilot_config", A.Config), ("pilot_stats", A.Stats)]:
        assert L.pilot_sizeof(name.encode()) == C.sizeof(cls), name
    assert L.pilot_sizeof(b"nope") == 0


def test_binding_constants_match_header():
    from paper_2606_31098_amd import _abi as A
    src = open(HEADER).read()
    for name, val in [("PILOT_EINVAL", A.EINVAL), ("PILOT_ENOMEM", A.ENOMEM), ("PILOT_EDEVICE", A.EDEVICE),
                      ("PILOT_EAGAIN", A.EAGAIN), ("PILOT_EUNSUPPORTED", A.EUNSUPPORTED),
                      ("PILOT_FLAG_NO_GRAPH", A.FLAG_NO_GRAPH), ("PILOT_FLAG_AUTOTUNE", A.FLAG_AUTOTUNE),
                      ("PILOT_FLAG_PROFILE", A.FLAG_PROFILE), ("PILOT_FLAG_KEEP_ORDER", A.FLAG_KEEP_ORDER),
                      ("PILOT_FLAG_SORT_ANCHORS", A.FLAG_SORT_ANCHORS)]:
        m = re.search(name + r"\s*=\s*(-?\d+)", src)
        assert m and int(m.group(1)) == val, name
    for name, val in [("PILOT_MAX_LEVELS", A.MAX_LEVELS)]:
        assert re.search(r"#define " + name + r"\s+(\d+)", src).group(1) == str(val)


def test_null_arguments_are_rejected_without_a_device(lib):
    from paper_2606_31098_amd import _abi as A
    L = A.load(LIB)
    assert L.pilot_create(None, None) == A.EINVAL
    assert b"out" in L.pilot_last_error(None)
    h = C.c_void_p()
    assert L.pilot_create(C.byref(h), None) == A.EINVAL
    assert h.value is None
    assert L.pilot_solve(None, None, 0, None) == A.EINVAL
    assert L.pilot_lift(None, None, 2, 2, 0.0, 0.0, 1.0, None, 1, None, 2, 2, 32, A.F32, 1.0,
                        None, None, None, None) == A.EINVAL
    L.pilot_destroy(None)


def test_product_path_has_no_oracle_dependency():
    """The binding and library never reference the CPU oracle."""
    pkg = os.path.join(ROOT, "paper_2606_31098_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".cpp", ".h", ".inc")):
                txt = open(os.path.join(dirpath, fn)).read()
                assert "import oracle" not in txt and "from oracle" not in txt and "liboracle" not in txt, fn
                assert "oracle.h" not in txt, fn


def test_bench_refuses_more_than_one_gpu():
    """bench.py --gpus N with N > 1 exits with a message (one GPU here)."""
    import json
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "--gpus must be 1" in json.loads(r.stdout.strip().splitlines()[-1])["error"]
